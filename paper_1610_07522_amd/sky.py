"""Thin Python binding of the C ABI in ``include/sky.h`` (ctypes).

Argument marshalling only: every step of the solver runs in ``libsky.so``.
Device memory (the context workspace and any state buffers) comes from
PyTorch tensors on a ROCm device; the library is handed raw pointers and the
current HIP stream.  Importing this module does not need a GPU; loading the
library does need the built ``libsky.so`` and raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsky.so")

SKY_OK = 0
SKY_NOT_CONVERGED = 1
SKY_ERR_INVALID = -1
SKY_ERR_UNSUPPORTED_GRID = -2
SKY_ERR_WORKSPACE = -3
SKY_ERR_HIP = -4
SKY_ERR_NOT_POSITIVE_DEFINITE = -5
SKY_ERR_NAN = -6
SKY_FP64 = 0
SKY_MIXED = 1
SKY_UPDATE_EXACT = 0
SKY_UPDATE_PAPER = 1
SKY_MAX_TWIST = 32

VIEW = dict(psi=0, hpsi=1, phi=2, hphi=3, dens=4, meanfield=5, coulomb=6, energy=7,
            eps=8, ritz=9, r2=10, overlap=11, hsub=12, evec=13, umat=14,
            pc_params=15, pc_grad=16, pc_samples=17, pc_gains=18)
_MATRIX_VIEWS = ("overlap", "hsub", "evec", "umat")
_F32_VIEWS = ("pc_params", "pc_grad", "pc_samples", "pc_gains")

# Symbols declared in include/sky.h, in order.
EXPORTS = ("sky_workspace_size", "sky_create", "sky_init_box", "sky_apply_h",
           "sky_apply_h_noalloc",
           "sky_damped_step", "sky_orthonormalize", "sky_densities", "sky_iterate",
           "sky_get_view", "sky_set_states", "sky_get_states", "sky_get_iteration",
           "sky_set_iteration", "sky_set_timing", "sky_get_timing", "sky_get_precision",
           "sky_autotune", "sky_get_tuning", "sky_set_graphs", "sky_batch_iterate",
           "sky_iterate_graph", "sky_batch_iterate_graph",
           "sky_precond_collect", "sky_precond_train",
           "sky_precond_loss_grad", "sky_precond_set_rows", "sky_precond_use",
           "sky_set_preconditioner", "sky_sync",
           "sky_last_error",
           "sky_destroy")
PHASES = ("apply_h", "damp", "overlap_gemm", "subspace", "combine_gemm", "densities",
          "meanfield", "split")


class BoxDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("dx", ctypes.c_double),
                ("n_neutrons", ctypes.c_int32), ("n_protons", ctypes.c_int32),
                ("t0", ctypes.c_double), ("t1", ctypes.c_double),
                ("t2", ctypes.c_double), ("t3", ctypes.c_double),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double),
                ("x2", ctypes.c_double), ("x3", ctypes.c_double),
                ("alpha", ctypes.c_double), ("W0", ctypes.c_double),
                ("hb2m_n", ctypes.c_double), ("hb2m_p", ctypes.c_double),
                ("e2", ctypes.c_double),
                ("damp_x0", ctypes.c_double), ("damp_e0", ctypes.c_double),
                ("precision", ctypes.c_int32), ("ladder_tol", ctypes.c_double),
                ("extra_n", ctypes.c_int32), ("extra_p", ctypes.c_int32),
                ("ntwist", ctypes.c_int32),
                ("twist", (ctypes.c_double * 3) * SKY_MAX_TWIST),
                ("update", ctypes.c_int32), ("one_h", ctypes.c_int32),
                ("dev_refine_steps", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("residual", ctypes.c_double),
                ("energy", ctypes.c_double), ("energy_per_a", ctypes.c_double),
                ("eig_iters", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("eig_fallbacks", ctypes.c_int32), ("precond_iters", ctypes.c_int32),
                ("eig_unconverged", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("h_lines", ctypes.c_int32), ("damp_xy", ctypes.c_int32),
                ("overlap_split", ctypes.c_int32 * 2), ("square_split", ctypes.c_int32 * 2),
                ("from_cache", ctypes.c_int32), ("overlap_waves", ctypes.c_int32 * 2),
                ("combine_waves", ctypes.c_int32 * 2)]

    def as_dict(self) -> Dict[str, object]:
        return dict(h_lines=self.h_lines, damp_xy=self.damp_xy,
                    overlap_split=list(self.overlap_split),
                    square_split=list(self.square_split), from_cache=bool(self.from_cache),
                    overlap_waves=list(self.overlap_waves),
                    combine_waves=list(self.combine_waves))


class SkyError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sky error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libsky.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} not found: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "sky_workspace_size": (ctypes.c_int, [ctypes.POINTER(BoxDesc), ctypes.POINTER(ctypes.c_size_t)]),
        "sky_create": (ctypes.c_int, [ctypes.POINTER(BoxDesc), vp, ctypes.c_size_t, vp,
                                      ctypes.POINTER(vp)]),
        "sky_init_box": (ctypes.c_int, [vp, vp, vp]),
        "sky_apply_h": (ctypes.c_int, [vp, i32, vp, vp, i32, vp]),
        "sky_apply_h_noalloc": (ctypes.c_int, [vp, i32, vp, vp, i32, vp]),
        "sky_damped_step": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, i32, vp]),
        "sky_orthonormalize": (ctypes.c_int, [vp, i32, vp, vp, vp, vp]),
        "sky_densities": (ctypes.c_int, [vp]),
        "sky_iterate": (ctypes.c_int, [vp, i32, dbl, ctypes.POINTER(Report)]),
        "sky_get_view": (ctypes.c_int, [vp, i32, i32, ctypes.POINTER(vp),
                                        ctypes.POINTER(ctypes.c_int64)]),
        "sky_set_states": (ctypes.c_int, [vp, i32, vp, i32]),
        "sky_get_states": (ctypes.c_int, [vp, i32, vp, i32]),
        "sky_get_iteration": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int64)]),
        "sky_set_iteration": (ctypes.c_int, [vp, ctypes.c_int64]),
        "sky_set_timing": (ctypes.c_int, [vp, i32]),
        "sky_get_timing": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int64)]),
        "sky_get_precision": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int32)]),
        "sky_autotune": (ctypes.c_int, [vp, ctypes.c_char_p, ctypes.POINTER(Tuning)]),
        "sky_get_tuning": (ctypes.c_int, [vp, ctypes.POINTER(Tuning)]),
        "sky_set_graphs": (ctypes.c_int, [vp, i32]),
        "sky_batch_iterate": (ctypes.c_int, [ctypes.POINTER(vp), i32, i32, i32, dbl,
                                             ctypes.POINTER(Report), ctypes.POINTER(ctypes.c_int32)]),
        "sky_iterate_graph": (ctypes.c_int, [vp, i32, dbl, i32, ctypes.POINTER(Report)]),
        "sky_batch_iterate_graph": (ctypes.c_int, [ctypes.POINTER(vp), i32, i32, i32, dbl, i32,
                                                   ctypes.POINTER(Report),
                                                   ctypes.POINTER(ctypes.c_int32)]),
        "sky_precond_collect": (ctypes.c_int, [vp, i32, ctypes.POINTER(ctypes.c_int32)]),
        "sky_precond_train": (ctypes.c_int, [vp, i32, dbl, dp]),
        "sky_precond_loss_grad": (ctypes.c_int, [vp, i32, dp]),
        "sky_precond_set_rows": (ctypes.c_int, [vp, i32]),
        "sky_precond_use": (ctypes.c_int, [vp, i32, dbl, i32]),
        "sky_set_preconditioner": (ctypes.c_int, [vp, vp, i32]),
        "sky_sync": (ctypes.c_int, [vp]),
        "sky_last_error": (ctypes.c_char_p, []),
        "sky_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _ = dp
    _lib = lib
    return lib


def _check(rc: int, ok=(SKY_OK,)) -> int:
    if rc not in ok:
        raise SkyError(rc, load().sky_last_error().decode())
    return rc


def desc_from_workload(w, precision: int = SKY_FP64, ladder_tol: float = 0.0,
                       twists=None, update: int = SKY_UPDATE_EXACT,
                       one_h: bool = False) -> BoxDesc:
    """BoxDesc of a ``paper_1610_07522_amd.inputs.Workload`` (its extra
    states included); ``twists``: Bloch phases (theta_x, theta_y, theta_z)
    of twist-averaged boundary conditions, None = periodic."""
    p = w.params
    d = BoxDesc(w.n, w.dx, w.n_neutrons, w.n_protons, p["t0"], p["t1"], p["t2"], p["t3"],
                p["x0"], p["x1"], p["x2"], p["x3"], p["alpha"], p["W0"],
                p["hb2m_n"], p["hb2m_p"], p["e2"], w.damp_x0, w.damp_e0,
                precision, ladder_tol)
    d.extra_n = getattr(w, "extra_n", 0)
    d.extra_p = getattr(w, "extra_p", 0)
    if twists:
        if len(twists) > SKY_MAX_TWIST:
            raise ValueError(f"at most {SKY_MAX_TWIST} twists")
        d.ntwist = len(twists)
        for t, th in enumerate(twists):
            for m in range(3):
                d.twist[t][m] = float(th[m])
    d.update = update
    d.one_h = 1 if one_h else 0
    return d


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _report_dict(rep: Report, rc: int) -> Dict[str, float]:
    return dict(iters=rep.iters, residual=rep.residual, energy=rep.energy,
                energy_per_a=rep.energy_per_a, eig_iters=rep.eig_iters,
                eig_fallbacks=rep.eig_fallbacks, precond_iters=rep.precond_iters,
                eig_unconverged=rep.eig_unconverged,
                precision=rep.precision, converged=(rc == SKY_OK))


def batch_iterate(boxes, nthreads: int, max_iter: int, tol: float = 0.0):
    """sky_batch_iterate over ``boxes`` (a list of Box): per-box report dicts."""
    if not boxes:
        return []
    lib = boxes[0].lib
    n = len(boxes)
    ctxs = (ctypes.c_void_p * n)(*[b.ctx.value for b in boxes])
    reps = (Report * n)()
    st = (ctypes.c_int32 * n)()
    _check(lib.sky_batch_iterate(ctxs, n, nthreads, max_iter, tol, reps, st))
    return [_report_dict(reps[i], st[i]) for i in range(n)]


def batch_iterate_graph(boxes, nthreads: int, max_iter: int, tol: float = 0.0, chunk: int = 16):
    """sky_batch_iterate_graph over ``boxes`` (a list of Box): per-box report dicts."""
    if not boxes:
        return []
    lib = boxes[0].lib
    n = len(boxes)
    ctxs = (ctypes.c_void_p * n)(*[b.ctx.value for b in boxes])
    reps = (Report * n)()
    st = (ctypes.c_int32 * n)()
    _check(lib.sky_batch_iterate_graph(ctxs, n, nthreads, max_iter, tol, chunk, reps, st))
    return [_report_dict(reps[i], st[i]) for i in range(n)]


class Box:
    """One solver context over a torch-allocated workspace on ``device``."""

    def __init__(self, desc: BoxDesc, device="cuda:0", stream=None):
        import torch
        self.lib = load()
        self.desc = desc
        self.device = torch.device(device)
        nbytes = ctypes.c_size_t()
        _check(self.lib.sky_workspace_size(ctypes.byref(desc), ctypes.byref(nbytes)))
        self.nbytes = nbytes.value
        self.ws = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._pad = (-base) % 256
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        ctx = ctypes.c_void_p()
        _check(self.lib.sky_create(ctypes.byref(desc), base + self._pad, self.nbytes,
                                   stream.cuda_stream, ctypes.byref(ctx)))
        self.ctx = ctx

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.sky_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- entry points
    def init_box(self, raw_n, raw_p):
        _check(self.lib.sky_init_box(self.ctx, _ptr(raw_n), _ptr(raw_p)))

    def apply_h(self, q, psi, hpsi, nstates, eps=None):
        _check(self.lib.sky_apply_h(self.ctx, q, _ptr(psi), _ptr(hpsi), nstates, _ptr(eps)))

    def apply_h_noalloc(self, q, psi, hpsi, nstates, eps=None):
        _check(self.lib.sky_apply_h_noalloc(self.ctx, q, _ptr(psi), _ptr(hpsi), nstates,
                                            _ptr(eps)))

    def damped_step(self, q, psi, hpsi, eps, phi, nstates, r2=None):
        _check(self.lib.sky_damped_step(self.ctx, q, _ptr(psi), _ptr(hpsi), _ptr(eps),
                                        _ptr(phi), nstates, _ptr(r2)))

    def orthonormalize(self, q, phi, hphi, psi_out, ritz=None):
        _check(self.lib.sky_orthonormalize(self.ctx, q, _ptr(phi), _ptr(hphi), _ptr(psi_out),
                                           _ptr(ritz)))

    def densities(self):
        _check(self.lib.sky_densities(self.ctx))

    @property
    def nsets(self) -> int:
        return 2 * max(1, self.desc.ntwist)

    def set_states(self, q, psi, precision=None):
        """Copy the states of set q from a device tensor (complex128 or complex64)."""
        import torch
        if precision is None:
            precision = SKY_MIXED if psi.dtype == torch.complex64 else SKY_FP64
        _check(self.lib.sky_set_states(self.ctx, q, _ptr(psi), precision))

    def get_states(self, q, out):
        """Copy the states of set q into a device tensor (complex128 or complex64)."""
        import torch
        precision = SKY_MIXED if out.dtype == torch.complex64 else SKY_FP64
        _check(self.lib.sky_get_states(self.ctx, q, _ptr(out), precision))

    def iteration(self) -> int:
        v = ctypes.c_int64()
        _check(self.lib.sky_get_iteration(self.ctx, ctypes.byref(v)))
        return v.value

    def set_iteration(self, it: int):
        _check(self.lib.sky_set_iteration(self.ctx, it))

    def iterate(self, max_iter: int, tol: float = 0.0) -> Dict[str, float]:
        rep = Report()
        rc = _check(self.lib.sky_iterate(self.ctx, max_iter, tol, ctypes.byref(rep)),
                    ok=(SKY_OK, SKY_NOT_CONVERGED))
        return _report_dict(rep, rc)

    def iterate_graph(self, max_iter: int, tol: float = 0.0, chunk: int = 16) -> Dict[str, float]:
        rep = Report()
        rc = _check(self.lib.sky_iterate_graph(self.ctx, max_iter, tol, chunk, ctypes.byref(rep)),
                    ok=(SKY_OK, SKY_NOT_CONVERGED))
        return _report_dict(rep, rc)

    def precision(self) -> int:
        p = ctypes.c_int32()
        _check(self.lib.sky_get_precision(self.ctx, ctypes.byref(p)))
        return p.value

    def autotune(self, cache_path: Optional[str] = None) -> Dict[str, object]:
        t = Tuning()
        p = cache_path.encode() if cache_path else None
        _check(self.lib.sky_autotune(self.ctx, p, ctypes.byref(t)))
        return t.as_dict()

    def tuning(self) -> Dict[str, object]:
        t = Tuning()
        _check(self.lib.sky_get_tuning(self.ctx, ctypes.byref(t)))
        return t.as_dict()

    def set_graphs(self, enable: bool):
        _check(self.lib.sky_set_graphs(self.ctx, 1 if enable else 0))

    def precond_collect(self, q: int) -> int:
        n = ctypes.c_int32()
        _check(self.lib.sky_precond_collect(self.ctx, q, ctypes.byref(n)))
        return n.value

    def precond_train(self, steps: int, lr: float = 1e-3) -> float:
        loss = ctypes.c_double()
        _check(self.lib.sky_precond_train(self.ctx, steps, lr, ctypes.byref(loss)))
        return loss.value

    def precond_loss_grad(self, nsamples: int) -> float:
        loss = ctypes.c_double()
        _check(self.lib.sky_precond_loss_grad(self.ctx, nsamples, ctypes.byref(loss)))
        return loss.value

    def precond_set_rows(self, nrows: int):
        _check(self.lib.sky_precond_set_rows(self.ctx, nrows))

    def precond_use(self, enable: bool, rise_tol: float = 0.05, retrain_every: int = 0):
        _check(self.lib.sky_precond_use(self.ctx, 1 if enable else 0, rise_tol, retrain_every))

    def set_preconditioner(self, params):
        """Load FP32 master parameters (a device tensor) into the learned damping."""
        _check(self.lib.sky_set_preconditioner(self.ctx, _ptr(params), params.numel()))

    def sync(self):
        _check(self.lib.sky_sync(self.ctx))

    def set_timing(self, enable: bool):
        _check(self.lib.sky_set_timing(self.ctx, 1 if enable else 0))

    def timing(self) -> Dict[str, Dict[str, float]]:
        """Per phase and species: accumulated device ms and launch counts."""
        n = 2 * len(PHASES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(self.lib.sky_get_timing(self.ctx, ms, cnt))
        return {p: dict(ms_n=ms[2 * i], ms_p=ms[2 * i + 1], launches_n=cnt[2 * i],
                        launches_p=cnt[2 * i + 1]) for i, p in enumerate(PHASES)}

    # -------------------------------------------------------------- views
    def view(self, what: str, q: int = 0):
        """A torch tensor aliasing one of the context's device buffers."""
        import torch
        ptr = ctypes.c_void_p()
        cnt = ctypes.c_int64()
        _check(self.lib.sky_get_view(self.ctx, VIEW[what], q, ctypes.byref(ptr),
                                     ctypes.byref(cnt)))
        is_state = what in ("psi", "hpsi", "phi", "hphi")
        is_cpx = is_state or what in _MATRIX_VIEWS
        dt = torch.complex128 if is_cpx else torch.float64
        esize = 16 if is_cpx else 8
        if is_state and self.precision() == SKY_MIXED:
            dt, esize = torch.complex64, 8
        if what in _F32_VIEWS:
            dt, esize = torch.float32, 4
        off = ptr.value - self.ws.data_ptr() if ptr.value else 0
        t = self.ws[off:off + cnt.value * esize].view(dt)
        n = self.desc.n
        if is_state:
            return t.view(-1, 2, n, n, n)
        if what in ("dens", "meanfield"):
            return t.view(-1, n, n, n)
        if what == "coulomb":
            return t.view(n, n, n)
        if what in _MATRIX_VIEWS:
            m = int(round(cnt.value ** 0.5))
            return t.view(m, m)
        if what == "pc_samples":
            return t.view(-1, 6)
        if what == "pc_gains":
            return t.view(-1, 8)
        return t
