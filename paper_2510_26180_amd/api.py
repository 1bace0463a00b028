"""Thin Python binding over the C ABI (include/klecgc.h).

Device memory and streams come from PyTorch (tensors on the context's GPU,
float64, contiguous); every step of the computation runs in the HIP library.
The functions keep the ABI's names and argument order.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import _lib as L


class KlecgcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{L.ERRORS.get(code, code)}: {msg}")
        self.code = code


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


@dataclass
class ProblemSpec:
    dim: int
    n: int
    T: float
    N: int
    J: int
    alpha: float
    forcing: float = 1.0
    precision: int = L.KC_PREC_F64
    tol: float = 1e-8
    max_iter: int = 60
    inner_rtol: float = 0.0
    inner_max_iter: int = 0
    cgc_rtol: float = 0.0
    cgc_max_iter: int = 0

    @property
    def Nx(self) -> int:
        return self.n ** self.dim

    @property
    def n_faces(self) -> int:
        return self.n + 1 if self.dim == 1 else 2 * self.n * (self.n + 1)

    def c(self) -> L.Problem:
        return L.Problem(self.dim, self.n, self.T, self.N, self.J, self.alpha, self.forcing,
                         self.precision, self.tol, self.max_iter, self.inner_rtol, self.inner_max_iter,
                         self.cgc_rtol, self.cgc_max_iter)

    @staticmethod
    def from_workload(w, **kw) -> "ProblemSpec":
        prec = L.KC_PREC_F64 if w.precision == "f64" else L.KC_PREC_F32_REFINED
        args = dict(dim=w.dim, n=w.n, T=w.T, N=w.N, J=w.J, alpha=w.alpha, forcing=w.forcing,
                    precision=prec, tol=w.tol, max_iter=w.max_iter)
        args.update(kw)
        return ProblemSpec(**args)


@dataclass
class ModelSpec:
    """One of the Section 5 model problems (klecgc_model)."""
    model: int
    n: int
    T: float
    N: int
    J: int
    alpha: float
    tol: float = 0.0
    max_iter: int = 30
    beta: float = 0.1
    newton_tol: float = 0.0
    newton_max_iter: int = 0

    @property
    def Nx(self) -> int:
        return self.n * self.n if self.model == L.KC_MODEL_ADE_P1 else self.n

    def c(self) -> L.Model:
        return L.Model(self.model, self.n, self.T, self.N, self.J, self.alpha, self.tol, self.max_iter,
                       self.beta, self.newton_tol, self.newton_max_iter)


class Handle:
    def __init__(self, ptr: int, free, **meta):
        self.ptr = ptr
        self._free = free
        self.__dict__.update(meta)

    def close(self):
        if self.ptr:
            self._free(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """klecgc_ctx bound to one device and a borrowed HIP stream."""

    def __init__(self, device: int = 0, stream=None):
        self.lib = L.load()
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        h = ctypes.c_void_p()
        rc = self.lib.klecgc_create(ctypes.byref(h), device, ctypes.c_void_p(stream))
        if rc != 0:
            raise KlecgcError(rc, "klecgc_create failed")
        self.h = h
        self.device = device

    def _check(self, rc: int, allow=()):
        if rc != 0 and rc not in allow:
            raise KlecgcError(rc, self.lib.klecgc_last_error(self.h).decode())
        return rc

    def last_stats(self) -> dict:
        out = (ctypes.c_int64 * 16)()
        self._check(self.lib.klecgc_last_stats(self.h, out))
        v = list(out)
        return {"fine_krylov_its": v[0], "fine_passes": v[1], "fine_solves": v[2], "fine_max_its": v[3],
                "cgc_krylov_its": v[4], "cgc_solves": v[6], "cgc_max_its": v[7],
                "fine_cycles": v[8], "fine_krylov_cycles": v[9], "fine_missed": v[10], "cgc_missed": v[11]}

    KCLASSES = ("fine", "shifted", "fft_fwd", "fft_inv", "defect", "gemm", "mlp")

    def last_times(self) -> dict:
        ms = (ctypes.c_double * 8)()
        cnt = (ctypes.c_int64 * 8)()
        self._check(self.lib.klecgc_last_times(self.h, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.KCLASSES)}

    # ---- tuning
    def set_tuning(self, n: int, fine_variant=-1, fine_pcg_rtol=1e-6, cgc_variant=-1, cgc_inner_rtol=1e-5,
                   mg_sweeps=0, mg_smoother=0):
        t = L.Tuning(fine_variant, fine_pcg_rtol, cgc_variant, cgc_inner_rtol, mg_sweeps, mg_smoother)
        self._check(self.lib.klecgc_set_tuning(self.h, n, ctypes.byref(t)))

    def get_tuning(self, n: int) -> dict:
        t = L.Tuning()
        self._check(self.lib.klecgc_get_tuning(self.h, n, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in L.Tuning._fields_}

    def autotune(self, prob: ProblemSpec, a) -> dict:
        t = L.Tuning()
        ms = (ctypes.c_double * 2)()
        pc = prob.c()
        self._check(self.lib.klecgc_autotune(self.h, ctypes.byref(pc), _ptr(a), a.shape[0], ctypes.byref(t), ms))
        out = {f: getattr(t, f) for f, _ in L.Tuning._fields_}
        out.update(fine_ms=ms[0], cgc_ms=ms[1])
        return out

    def close(self):
        if getattr(self, "h", None):
            self.lib.klecgc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- KL / gPC
    def kle_build_field(self, dim: int, n: int, d: int, corr_len: float, sigma: float) -> Handle:
        desc = L.KleDesc(L.KC_KLE_FIELD_EXP, dim, n, d, corr_len, sigma, 0, 0.0)
        out = ctypes.c_void_p()
        nm = ctypes.c_int32()
        self._check(self.lib.kle_build(self.h, ctypes.byref(desc), None, 0, ctypes.byref(out), ctypes.byref(nm)))
        return Handle(out.value, self.lib.klecgc_kle_free, d=nm.value, dim=dim, n=n)

    def kle_build(self, S, eps_kl: float) -> Handle:
        n_t, Lrow = S.shape
        desc = L.KleDesc(L.KC_KLE_SNAPSHOT, 0, 0, 0, 0.0, 0.0, Lrow, eps_kl)
        out = ctypes.c_void_p()
        nm = ctypes.c_int32()
        self._check(self.lib.kle_build(self.h, ctypes.byref(desc), _ptr(S), n_t, ctypes.byref(out), ctypes.byref(nm)))
        return Handle(out.value, self.lib.klecgc_kle_free, n_modes=nm.value, L=Lrow, n_t=n_t)

    def kle_synthesize(self, field: Handle, xi, a, a32=None):
        self._check(self.lib.kle_synthesize(self.h, field.ptr, _ptr(xi), xi.shape[0], _ptr(a), _ptr(a32)))
        return a

    def kle_export(self, snap: Handle, mean=None, W=None, lam=None):
        self._check(self.lib.kle_export(self.h, snap.ptr, _ptr(mean), _ptr(W), _ptr(lam)))

    def gpc_fit(self, snap: Handle, xi_train, p: int, basis: int = L.KC_GPC_HERMITE) -> Handle:
        n_t, d = xi_train.shape
        out = ctypes.c_void_p()
        P = ctypes.c_int32()
        self._check(self.lib.gpc_fit(self.h, snap.ptr, _ptr(xi_train), n_t, d, p, basis, ctypes.byref(out),
                                     ctypes.byref(P)))
        return Handle(out.value, self.lib.klecgc_gpc_free, P=P.value, d=d, p=p, snap=snap)

    def gpc_predict(self, gpc: Handle, xi, U0):
        self._check(self.lib.gpc_predict(self.h, gpc.ptr, _ptr(xi), xi.shape[0], _ptr(U0)))
        return U0

    # ---- parareal pieces
    def fine_propagate(self, prob: ProblemSpec, a, start, end, allow_noconv=False, active=None) -> int:
        pc = prob.c()
        return self._check(self.lib.fine_propagate(self.h, ctypes.byref(pc), _ptr(a), _ptr(start), start.shape[0],
                                                   _ptr(end), _ptr(active)),
                           allow=(-5,) if allow_noconv else ())

    def fine_propagate_noalloc(self, prob: ProblemSpec, a, start, end, allow_noconv=False, active=None) -> int:
        pc = prob.c()
        return self._check(self.lib.fine_propagate_noalloc(self.h, ctypes.byref(pc), _ptr(a), _ptr(start),
                                                           start.shape[0], _ptr(end), _ptr(active)),
                           allow=(-5,) if allow_noconv else ())

    def cgc_diag_solve(self, prob: ProblemSpec, a, r, u, allow_noconv=False) -> int:
        pc = prob.c()
        return self._check(self.lib.cgc_diag_solve(self.h, ctypes.byref(pc), _ptr(a), _ptr(r), r.shape[0], _ptr(u)),
                           allow=(-5,) if allow_noconv else ())

    def serial_fine_propagate(self, prob: ProblemSpec, a, u0, U, allow_noconv=False) -> int:
        pc = prob.c()
        return self._check(self.lib.serial_fine_propagate(self.h, ctypes.byref(pc), _ptr(a), _ptr(u0), U.shape[0], _ptr(U)),
                           allow=(-5,) if allow_noconv else ())

    def coarse_propagate(self, prob: ProblemSpec, a, u0, U) -> int:
        pc = prob.c()
        return self._check(self.lib.coarse_propagate(self.h, ctypes.byref(pc), _ptr(a), _ptr(u0), U.shape[0], _ptr(U)))

    def parareal_solve(self, prob: ProblemSpec, a, U, u0=None, init: int = L.KC_INIT_ZERO, init_U=None,
                       gpc: Optional[Handle] = None, xi=None, allow_noconv=False, mlp: Optional[Handle] = None,
                       seed: int = 0, guess_out: Optional[np.ndarray] = None):
        """Returns (iters, status, increment history, rc); guess_out [M] int32 (optional)
        receives the guess each sample started from."""
        M = U.shape[0]
        iters = (ctypes.c_int32 * M)()
        status = (ctypes.c_int32 * M)()
        hist = (ctypes.c_double * (M * prob.max_iter))()
        guess = (ctypes.c_int32 * M)()
        pc = prob.c()
        rc = self.lib.parareal_solve(self.h, ctypes.byref(pc), _ptr(a), _ptr(u0), M, init, _ptr(init_U),
                                     gpc.ptr if gpc is not None else None, mlp.ptr if mlp is not None else None,
                                     _ptr(xi), ctypes.c_uint64(seed), _ptr(U), iters, status, hist, guess)
        self._check(rc, allow=(-5,) if allow_noconv else ())
        if guess_out is not None:
            guess_out[:] = np.frombuffer(guess, dtype=np.int32)
        return (np.frombuffer(iters, dtype=np.int32).copy(), np.frombuffer(status, dtype=np.int32).copy(),
                np.frombuffer(hist, dtype=np.float64).reshape(M, prob.max_iter).copy(), rc)

    def parareal_solve_sequential(self, prob: ProblemSpec, a, U, u0=None, init: int = L.KC_INIT_ZERO, init_U=None,
                                  gpc: Optional[Handle] = None, xi=None, mlp: Optional[Handle] = None, seed: int = 0,
                                  allow_noconv=False):
        """Algorithm 1 (sequential coarse grid correction); returns (iters, status, increments, rc)."""
        M = U.shape[0]
        iters = (ctypes.c_int32 * M)()
        status = (ctypes.c_int32 * M)()
        hist = (ctypes.c_double * (M * prob.max_iter))()
        pc = prob.c()
        rc = self.lib.parareal_solve_sequential(self.h, ctypes.byref(pc), _ptr(a), _ptr(u0), M, init, _ptr(init_U),
                                                gpc.ptr if gpc is not None else None,
                                                mlp.ptr if mlp is not None else None, _ptr(xi),
                                                ctypes.c_uint64(seed), _ptr(U), iters, status, hist)
        self._check(rc, allow=(-5,) if allow_noconv else ())
        return (np.frombuffer(iters, dtype=np.int32).copy(), np.frombuffer(status, dtype=np.int32).copy(),
                np.frombuffer(hist, dtype=np.float64).reshape(M, prob.max_iter).copy(), rc)

    # ---- Section 5 model problems ------------------------------------------------------
    def model_fine_propagate(self, mp: ModelSpec, c, start, end):
        pc = mp.c()
        return self._check(self.lib.model_fine_propagate(self.h, ctypes.byref(pc), _ptr(c), _ptr(start),
                                                         start.shape[0], _ptr(end)))

    def model_coarse_propagate(self, mp: ModelSpec, c, U, u0=None):
        pc = mp.c()
        return self._check(self.lib.model_coarse_propagate(self.h, ctypes.byref(pc), _ptr(c), _ptr(u0), U.shape[0],
                                                           _ptr(U)))

    def model_serial_fine(self, mp: ModelSpec, c, U, u0=None):
        pc = mp.c()
        return self._check(self.lib.model_serial_fine(self.h, ctypes.byref(pc), _ptr(c), _ptr(u0), U.shape[0],
                                                      _ptr(U)))

    def model_cgc_solve(self, mp: ModelSpec, c, Uk, F, Unew):
        M = Uk.shape[0]
        its = (ctypes.c_int32 * M)()
        pc = mp.c()
        self._check(self.lib.model_cgc_solve(self.h, ctypes.byref(pc), _ptr(c), _ptr(Uk), _ptr(F), M, _ptr(Unew), its))
        return np.frombuffer(its, dtype=np.int32).copy()

    def model_parareal_solve(self, mp: ModelSpec, c, U, u0=None, init: int = L.KC_INIT_ZERO, init_U=None,
                             gpc: Optional[Handle] = None, xi=None, seed: int = 0, ref=None,
                             sequential: bool = False):
        """Algorithms 2/3 (or Algorithm 1 with sequential=True) for a model problem; returns
        (iters, status, increments [M][max_iter], errors [M][max_iter+1][N] or None)."""
        M = U.shape[0]
        iters = (ctypes.c_int32 * M)()
        status = (ctypes.c_int32 * M)()
        hist = (ctypes.c_double * (M * mp.max_iter))()
        err = (ctypes.c_double * (M * (mp.max_iter + 1) * mp.N))() if ref is not None else None
        pc = mp.c()
        fn = self.lib.model_parareal_solve_sequential if sequential else self.lib.model_parareal_solve
        self._check(fn(self.h, ctypes.byref(pc), _ptr(c), _ptr(u0), M, init, _ptr(init_U),
                       gpc.ptr if gpc is not None else None, _ptr(xi), ctypes.c_uint64(seed), _ptr(ref), _ptr(U),
                       iters, status, hist, err))
        errs = (np.frombuffer(err, dtype=np.float64).reshape(M, mp.max_iter + 1, mp.N).copy()
                if err is not None else None)
        return (np.frombuffer(iters, dtype=np.int32).copy(), np.frombuffer(status, dtype=np.int32).copy(),
                np.frombuffer(hist, dtype=np.float64).reshape(M, mp.max_iter).copy(), errs)

    def parareal_solve_batch(self, base: ProblemSpec, tasks, a, U, init: int = L.KC_INIT_ZERO, graph: bool = True,
                             allow_noconv=False, progress: bool = False, persistent: bool = False):
        """tasks: sequence of (n, N, face_off, state_off); a, U: flat float64 device buffers."""
        M = len(tasks)
        arr = (L.Task * M)(*[L.Task(int(n), int(N), int(fo), int(so)) for n, N, fo, so in tasks])
        iters = (ctypes.c_int32 * M)()
        status = (ctypes.c_int32 * M)()
        lat = (ctypes.c_double * M)()
        total = ctypes.c_double()
        pc = base.c()
        rc = self.lib.parareal_solve_batch(self.h, ctypes.byref(pc), arr, M, _ptr(a), init, _ptr(U),
                                           (L.KC_BATCH_GRAPH if graph else 0) |
                                           (L.KC_BATCH_PROGRESS if progress else 0) |
                                           (L.KC_BATCH_PERSISTENT if persistent else 0), iters, status, lat,
                                           ctypes.byref(total))
        self._check(rc, allow=(-5,) if allow_noconv else ())
        return (np.frombuffer(iters, dtype=np.int32).copy(), np.frombuffer(status, dtype=np.int32).copy(),
                np.frombuffer(lat, dtype=np.float64).copy(), total.value, rc)

    # ---- learned initial guess
    def mlp_create(self, n_in: int, hidden: int, n_out: int, params=None) -> Handle:
        out = ctypes.c_void_p()
        npar = ctypes.c_int64()
        self._check(self.lib.mlp_create(self.h, n_in, hidden, n_out, ctypes.byref(out), ctypes.byref(npar)))
        h = Handle(out.value, self.lib.klecgc_mlp_free, n_in=n_in, hidden=hidden, n_out=n_out, n_params=npar.value)
        if params is not None:
            self.mlp_set_params(h, params)
        return h

    def mlp_set_params(self, h: Handle, params):
        self._check(self.lib.mlp_set_params(self.h, h.ptr, _ptr(params)))

    def mlp_get_params(self, h: Handle, params=None, mean=None, std=None):
        self._check(self.lib.mlp_get_params(self.h, h.ptr, _ptr(params), _ptr(mean), _ptr(std)))

    def mlp_normalize_targets(self, h: Handle, Y):
        self._check(self.lib.mlp_normalize_targets(self.h, h.ptr, _ptr(Y), Y.shape[0]))
        return Y

    def mlp_train(self, h: Handle, xi, Y, epochs: int, batch: int, lr: float, perm=None,
                  lr_final: float = 0.0) -> np.ndarray:
        loss = (ctypes.c_float * max(epochs, 1))()
        self._check(self.lib.mlp_train(self.h, h.ptr, _ptr(xi), _ptr(Y), xi.shape[0], epochs, batch, lr, lr_final,
                                       _ptr(perm), loss))
        return np.frombuffer(loss, dtype=np.float32)[:epochs].copy()

    def mlp_predict(self, h: Handle, xi, Y):
        self._check(self.lib.mlp_predict(self.h, h.ptr, _ptr(xi), xi.shape[0], _ptr(Y)))
        return Y

    def mlp_grad(self, h: Handle, xi, Y, grads) -> float:
        loss = ctypes.c_double()
        self._check(self.lib.mlp_grad(self.h, h.ptr, _ptr(xi), _ptr(Y), xi.shape[0], _ptr(grads), ctypes.byref(loss)))
        return loss.value

    def grid_restrict(self, n: int, nc: int, U, Yc):
        R = U.numel() // (n * n)
        self._check(self.lib.grid_restrict(self.h, n, nc, _ptr(U), R, _ptr(Yc)))
        return Yc

    def mlp_initial_guess(self, h: Handle, n: int, nc: int, N: int, xi, U0):
        self._check(self.lib.mlp_initial_guess(self.h, h.ptr, n, nc, N, _ptr(xi), xi.shape[0], _ptr(U0)))
        return U0
