"""MI355X Gaussian Belief Propagation for bundle adjustment.

Thin Python binding of the C ABI in include/gbp.h. The binding only marshals
arguments: every step of the GBP sweep (relinearisation, factor messages,
beliefs, reprojection statistics) runs in the HIP library libgbp_hip.so.
PyTorch provides the device workspace and the stream. There is no CPU
fallback: without the built library or a GPU the constructor raises.
"""
from __future__ import annotations

import ctypes as C
from typing import Sequence

import numpy as np

from . import _capi
from ._capi import (GBP_FP32, GBP_FP64, GBP_DAMP_ETA, GBP_DAMP_ETA_LAMBDA,
                    HipLibraryMissing, gbp_reproj)

__all__ = ["GBPSolver", "GBPError", "GBP_FP32", "GBP_FP64", "GBP_DAMP_ETA",
           "GBP_DAMP_ETA_LAMBDA", "HipLibraryMissing", "load_library"]


class GBPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_capi.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load_library():
    return _capi.load()


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


class GBPSolver:
    """One GBP problem, or a batch of independent problems run as one graph.

    `problems` is one object or a sequence of objects with attributes
    factor_kf, factor_lm, kf_init, lm_init, kf_anchor_info, z and cam
    (fx, fy, cx, cy, sigma)."""

    def __init__(self, problems, *, precision: int = GBP_FP32,
                 damp_mode: int = GBP_DAMP_ETA, beta: float = 0.01,
                 relin_interval: int = 10, undamped: int = 8,
                 anneal: bool | None = None, anneal_iters: int = 10,
                 weaken: float = 0.01, huber_k: float = 2.0, zmin: float = 1e-3,
                 capacity: tuple | None = None, device: int = 0,
                 use_torch: bool = True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("GBPSolver needs a ROCm GPU (torch.cuda is not available)")
        self._lib = _capi.load()
        self._torch = torch
        single = not isinstance(problems, (list, tuple))
        probs: Sequence = [problems] if single else list(problems)
        self.n_problems = len(probs)
        self._keep = []
        n = len(probs)
        graphs = (_capi.gbp_graph * n)()
        cams = (_capi.gbp_camera * n)()
        meas = (_capi.gbp_measurements * n)()
        self.kf_counts, self.lm_counts, self.f_counts = [], [], []
        for i, p in enumerate(probs):
            fkf, flm = _i32(p.factor_kf), _i32(p.factor_lm)
            kfi, lmi = _f64(p.kf_init), _f64(p.lm_init)
            anc = _f64(p.kf_anchor_info) if p.kf_anchor_info is not None else None
            z = _f64(p.z)
            self._keep += [fkf, flm, kfi, lmi, anc, z]
            nk, nl, nf = kfi.shape[0], lmi.shape[0], fkf.shape[0]
            graphs[i] = _capi.gbp_graph(nk, nl, nf, _ptr(fkf, C.c_int32), _ptr(flm, C.c_int32),
                                        _ptr(kfi, C.c_double), _ptr(lmi, C.c_double),
                                        _ptr(anc, C.c_double))
            c = p.cam
            cams[i] = _capi.gbp_camera(c.fx, c.fy, c.cx, c.cy, c.sigma)
            meas[i] = _capi.gbp_measurements(_ptr(z, C.c_double))
            self.kf_counts.append(nk)
            self.lm_counts.append(nl)
            self.f_counts.append(nf)
        opt = _capi.gbp_options()
        self._lib.gbp_default_options(C.byref(opt))
        opt.precision = precision
        opt.damp_mode = damp_mode
        opt.beta = beta
        opt.relin_min_interval = relin_interval
        opt.undamped_after_relin = undamped
        opt.anneal = int(precision == GBP_FP32) if anneal is None else int(anneal)
        opt.prior_anneal_iters = anneal_iters
        opt.prior_weaken = weaken
        opt.huber_k = huber_k
        opt.zmin = zmin
        if capacity is not None:
            opt.max_keyframes, opt.max_landmarks, opt.max_factors = capacity
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        # a dedicated stream (HIP graphs cannot be captured on the null stream)
        self.stream = torch.cuda.Stream(device=self.device)
        opt.stream = C.c_void_p(self.stream.cuda_stream)
        self.workspace = None
        if use_torch:
            nbytes = C.c_size_t(0)
            self._check(self._lib.gbp_workspace_bytes(n, graphs, C.byref(opt), C.byref(nbytes)), None)
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            opt.workspace = C.c_void_p(self.workspace.data_ptr())
            opt.workspace_bytes = nbytes.value
        torch.cuda.current_stream(self.device).synchronize()
        self.h = C.c_void_p()
        if single:
            st = self._lib.gbp_create(graphs, cams, meas, C.byref(opt), C.byref(self.h))
        else:
            st = self._lib.gbp_create_batch(n, graphs, cams, meas, C.byref(opt), C.byref(self.h))
        self._check(st, self.h)
        self.precision = precision
        self.huber_k = huber_k
        self._keep_opt = opt

    # ------------------------------------------------------------------
    def _check(self, st, h):
        if st != 0:
            msg = self._lib.gbp_last_error(h).decode() if h is not None and h.value else ""
            raise GBPError(st, msg)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self._lib.gbp_destroy(self.h)
            self.h = C.c_void_p()
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def sizes(self):
        v = [C.c_int32() for _ in range(5)]
        self._check(self._lib.gbp_sizes(self.h, *[C.byref(x) for x in v]), self.h)
        return tuple(x.value for x in v)

    @property
    def last_relinearised(self) -> int:
        """Factors relinearised in the most recent iteration."""
        v = C.c_int64(0)
        self._check(self._lib.gbp_counters(self.h, C.byref(v)), self.h)
        return v.value

    @property
    def t(self) -> int:
        return self.sizes[4]

    # ------------------------------------------------------------------
    def relinearise(self, beta: float = -1.0) -> int:
        n = C.c_int32(0)
        self._check(self._lib.gbp_relinearise(self.h, float(beta), C.byref(n)), self.h)
        return n.value

    def iterate(self, n: int, damping: float = 0.4, huber_k: float | None = None) -> None:
        if huber_k is not None:
            self.huber_k = huber_k
        self._check(self._lib.gbp_iterate(self.h, int(n), float(damping), float(self.huber_k)), self.h)

    def iterate_logged(self, n: int, damping: float = 0.4, huber_k: float | None = None,
                       log_every: int = 1) -> np.ndarray:
        """Returns [n // log_every, n_problems, 4] rows of (t, are_all, are_ref, n_linear)."""
        if huber_k is not None:
            self.huber_k = huber_k
        rows = n // log_every
        out = np.zeros((max(rows, 1), self.n_problems, 4))
        self._check(self._lib.gbp_iterate_logged(self.h, int(n), float(damping), float(self.huber_k),
                                                 int(log_every), _ptr(out, C.c_double)), self.h)
        return out[:rows]

    def phase_times(self, n: int, damping: float = 0.4, huber_k: float | None = None) -> dict:
        """Average ms per launch of each phase over n real iterations."""
        if huber_k is not None:
            self.huber_k = huber_k
        ms = np.zeros(5)
        self._check(self._lib.gbp_phase_times(self.h, int(n), float(damping), float(self.huber_k),
                                              _ptr(ms, C.c_double)), self.h)
        return dict(check=ms[0], relin=ms[1], factor_kf=ms[2], belief_lm=ms[3], reproj=ms[4])

    def autotune(self, n_iters: int = 5, cache_path: str | None = None) -> tuple:
        """Pick workgroup sizes by timing (state restored); returns (kf, lm)."""
        chosen = (C.c_int32 * 2)()
        path = cache_path.encode() if cache_path else None
        self._check(self._lib.gbp_autotune(self.h, int(n_iters), path, chosen), self.h)
        return chosen[0], chosen[1]

    def synchronize(self):
        self.stream.synchronize()

    def beliefs(self, info: bool = False) -> dict:
        nk, nl = sum(self.kf_counts), sum(self.lm_counts)
        kf = np.zeros((nk, 6))
        lm = np.zeros((nl, 3))
        ki = np.zeros((nk, 6, 6)) if info else None
        li = np.zeros((nl, 3, 3)) if info else None
        self._check(self._lib.gbp_beliefs(self.h, _ptr(kf, C.c_double), _ptr(lm, C.c_double),
                                          _ptr(ki, C.c_double), _ptr(li, C.c_double)), self.h)
        out = dict(kf_mu=kf, lm_mu=lm)
        if info:
            out.update(kf_lam=ki, lm_lam=li)
        return out

    def reproj(self, problem_index: int = -1) -> dict:
        r = gbp_reproj()
        self._check(self._lib.gbp_reproj_stats(self.h, int(problem_index), C.byref(r)), self.h)
        return dict(are_all=r.are_all, are_quadratic=r.are_quadratic, are_ref=r.are_ref,
                    n_valid=r.n_valid, n_quadratic=r.n_quadratic, n_linear=r.n_linear,
                    n_invalid=r.n_invalid, n_ref=r.n_ref)

    def reproj_error(self):
        a, q, n = C.c_double(), C.c_double(), C.c_int32()
        self._check(self._lib.gbp_reproj_error(self.h, C.byref(a), C.byref(q), C.byref(n)), self.h)
        return a.value, q.value, n.value

    def set_reference(self, z_ref, mask) -> None:
        if z_ref is None:
            self._check(self._lib.gbp_set_reference(self.h, None, None), self.h)
            return
        zr = _f64(z_ref)
        mk = np.ascontiguousarray(mask, dtype=np.uint8)
        self._check(self._lib.gbp_set_reference(self.h, _ptr(zr, C.c_double),
                                                _ptr(mk, C.c_uint8)), self.h)

    def add_keyframe(self, pose, lm_init, f_kf, f_lm, z) -> None:
        pose = None if pose is None else _f64(pose, (6,))
        lmi = _f64(lm_init).reshape(-1, 3)
        fk, fl = _i32(f_kf), _i32(f_lm)
        zz = _f64(z).reshape(-1, 2)
        self._check(self._lib.gbp_add_keyframe(self.h, _ptr(pose, C.c_double), lmi.shape[0],
                                               _ptr(lmi, C.c_double), fk.shape[0],
                                               _ptr(fk, C.c_int32), _ptr(fl, C.c_int32),
                                               _ptr(zz, C.c_double)), self.h)
        if pose is not None:
            self.kf_counts[-1] += 1
        self.lm_counts[-1] += lmi.shape[0]
        self.f_counts[-1] += fk.shape[0]

    def set_damping_model(self, weights_bf16: np.ndarray | None, every_k: int = 5) -> None:
        if weights_bf16 is None:
            self._check(self._lib.gbp_set_damping_model(self.h, None, 0), self.h)
            return
        w = np.ascontiguousarray(weights_bf16, dtype=np.uint16)
        self._keep_w = w
        self._check(self._lib.gbp_set_damping_model(self.h, _ptr(w, C.c_uint16), int(every_k)), self.h)
