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
                    GBP_PAIR_KEYFRAMES, GBP_PAIR_LANDMARKS, GBP_PAIR_ODOMETRY, HipLibraryMissing,
                    GBP_OK, GBP_EINVAL, GBP_ENOMEM, GBP_EDEVICE, GBP_ENUMERIC, GBP_ESTATE,
                    gbp_reproj)

__all__ = ["GBPSolver", "GBPError", "GBP_FP32", "GBP_FP64", "GBP_DAMP_ETA",
           "GBP_DAMP_ETA_LAMBDA", "GBP_PAIR_KEYFRAMES", "GBP_PAIR_LANDMARKS", "GBP_PAIR_ODOMETRY", "HipLibraryMissing", "load_library", "mlp_infer",
           "MLPTrainer", "MLP_PARAMS", "MLP_FEATURES", "GBP_OK", "GBP_EINVAL", "GBP_ENOMEM",
           "GBP_EDEVICE", "GBP_ENUMERIC", "GBP_ESTATE"]

MLP_PARAMS = _capi.MLP_PARAMS
MLP_FEATURES = _capi.MLP_FEATURES
LOG_COLS = _capi.LOG_COLS


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
            # the library reads exactly these sizes from each array
            if (fkf.shape != (nf,) or flm.shape != (nf,) or z.shape != (nf, 2) or kfi.shape != (nk, 6)
                    or lmi.shape != (nl, 3) or (anc is not None and anc.shape != (nk,))):
                raise ValueError(f"problem {i}: need factor_kf, factor_lm [nf], z [nf, 2], kf_init [nk, 6], "
                                 f"lm_init [nl, 3] and kf_anchor_info [nk] or None")
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

    def _huber(self, huber_k):
        # the threshold to pass: the new one, else the last one accepted
        return float(self.huber_k if huber_k is None else huber_k)

    def iterate(self, n: int, damping: float = 0.4, huber_k: float | None = None) -> None:
        hk = self._huber(huber_k)
        self._check(self._lib.gbp_iterate(self.h, int(n), float(damping), hk), self.h)
        self.huber_k = hk

    def iterate_logged(self, n: int, damping: float = 0.4, huber_k: float | None = None,
                       log_every: int = 1) -> np.ndarray:
        """Returns [n // log_every, n_problems, 5] rows of (t, are_all, are_ref,
        n_linear, n_linear_ref)."""
        hk = self._huber(huber_k)
        rows = n // log_every if log_every >= 1 else 0  # the library refuses log_every < 1
        out = np.zeros((max(rows, 1), self.n_problems, LOG_COLS))
        self._check(self._lib.gbp_iterate_logged(self.h, int(n), float(damping), hk,
                                                 int(log_every), _ptr(out, C.c_double)), self.h)
        self.huber_k = hk
        return out[:rows]

    def phase_times(self, n: int, damping: float = 0.4, huber_k: float | None = None) -> dict:
        """Average ms per launch of each phase over n real iterations."""
        hk = self._huber(huber_k)
        ms = np.zeros(6)
        self._check(self._lib.gbp_phase_times(self.h, int(n), float(damping), hk,
                                              _ptr(ms, C.c_double)), self.h)
        self.huber_k = hk
        return dict(check=ms[0], relin=ms[1], factor_kf=ms[2], belief_lm=ms[3], reproj=ms[4],
                    k_factor_kf=ms[5])

    def autotune(self, n_iters: int = 5, cache_path: str | None = None) -> tuple:
        """Pick workgroup sizes, lanes per landmark, where the keyframe
        solves run and relinearisation segments per workgroup by timing
        (state restored); returns (kf block, lm block, lanes per landmark,
        relinearisation segments, keyframe solves fused into the landmark
        launch: 1 or 0)."""
        chosen = (C.c_int32 * 5)()
        path = cache_path.encode() if cache_path else None
        self._check(self._lib.gbp_autotune(self.h, int(n_iters), path, chosen), self.h)
        return tuple(int(v) for v in chosen)

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
                    n_invalid=r.n_invalid, n_ref=r.n_ref, n_linear_ref=r.n_linear_ref)

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
        nf = sum(self.f_counts)
        if zr.shape != (nf, 2) or mk.shape != (nf,):
            raise ValueError(f"set_reference: need z_ref [{nf}, 2] and mask [{nf}] (every factor of the batch)")
        self._check(self._lib.gbp_set_reference(self.h, _ptr(zr, C.c_double),
                                                _ptr(mk, C.c_uint8)), self.h)

    def add_pair_factors(self, kind: int, a, b, z, precision) -> None:
        """Pairwise difference factors x_b - x_a ~ N(z, diag(precision)^-1)
        between keyframes (GBP_PAIR_KEYFRAMES, 6 values per factor) or
        landmarks (GBP_PAIR_LANDMARKS, 3 values), or odometry factors on the
        camera centres of two keyframes (GBP_PAIR_ODOMETRY, 3 values);
        indices in the caller's order (problem-major for batches)."""
        D = 6 if kind == GBP_PAIR_KEYFRAMES else 3
        a_, b_ = _i32(np.asarray(a).ravel()), _i32(np.asarray(b).ravel())
        z_ = _f64(np.asarray(z, dtype=np.float64).reshape(-1, D))
        p_ = _f64(np.asarray(precision, dtype=np.float64).reshape(-1, D))
        if not (a_.shape[0] == b_.shape[0] == z_.shape[0] == p_.shape[0]):
            raise ValueError("a, b, z and precision need one entry per factor")
        self._check(self._lib.gbp_add_pair_factors(self.h, int(kind), a_.shape[0], _ptr(a_, C.c_int32),
                                                   _ptr(b_, C.c_int32), _ptr(z_, C.c_double),
                                                   _ptr(p_, C.c_double)), self.h)

    def add_keyframe(self, pose, lm_init, f_kf, f_lm, z) -> None:
        pose = None if pose is None else _f64(pose, (6,))
        lmi = _f64(lm_init).reshape(-1, 3)
        fk, fl = _i32(f_kf), _i32(f_lm)
        zz = _f64(z).reshape(-1, 2)
        if fk.ndim != 1 or fl.shape != fk.shape or zz.shape[0] != fk.shape[0]:
            raise ValueError("add_keyframe: f_kf, f_lm and z need one entry per new factor")
        self._check(self._lib.gbp_add_keyframe(self.h, _ptr(pose, C.c_double), lmi.shape[0],
                                               _ptr(lmi, C.c_double), fk.shape[0],
                                               _ptr(fk, C.c_int32), _ptr(fl, C.c_int32),
                                               _ptr(zz, C.c_double)), self.h)
        if pose is not None:
            self.kf_counts[-1] += 1
        self.lm_counts[-1] += lmi.shape[0]
        self.f_counts[-1] += fk.shape[0]

    def set_damping_model(self, weights_bf16: np.ndarray | None, every_k: int = 5,
                          fallback_rise: float = 0.1) -> None:
        """Switch the learned per-factor damping on (BF16 bit patterns of
        the network parameters) or off (None)."""
        if weights_bf16 is None:
            self._check(self._lib.gbp_set_damping_model(self.h, None, 0, 0.0), self.h)
            return
        w = np.ascontiguousarray(weights_bf16, dtype=np.uint16)
        if w.shape != (_capi.MLP_PARAMS,):
            raise ValueError(f"weights must have {_capi.MLP_PARAMS} entries")
        self._keep_w = w
        self._check(self._lib.gbp_set_damping_model(self.h, _ptr(w, C.c_uint16), int(every_k),
                                                     float(fallback_rise)), self.h)

    def set_damping_judges(self, judge_of) -> None:
        """Plain GBP as the judge of the learned damping: judge_of[i] = j names
        problem j of the batch (the same problem, run with the constant
        damping) as problem i's judge; -1: the best-seen rule; None: no
        judges. Call after set_damping_model."""
        if judge_of is None:
            self._check(self._lib.gbp_set_damping_judges(self.h, None), self.h)
            return
        j = _i32(judge_of).ravel()
        if j.size != self.n_problems:
            raise ValueError("one judge entry per problem")
        self._check(self._lib.gbp_set_damping_judges(self.h, _ptr(j, C.c_int32)), self.h)

    def reset(self) -> None:
        """Back to the state right after creation (keeps recorded graphs)."""
        self._check(self._lib.gbp_reset(self.h), self.h)

    def apply_depth_model(self, landmarks) -> None:
        """Move the listed landmarks (caller indices) by the network's
        log-depth head along their newest keyframe's ray and restart their
        factors there."""
        lm = _i32(landmarks).ravel()
        self._check(self._lib.gbp_apply_depth_model(self.h, _ptr(lm, C.c_int32), int(lm.size)), self.h)

    def fallback_flags(self) -> np.ndarray:
        out = np.zeros(self.n_problems, dtype=np.int32)
        self._check(self._lib.gbp_fallback_flags(self.h, _ptr(out, C.c_int32)), self.h)
        return out

    def _device_rows(self, fn, idx, width):
        # buffers belong to torch's current stream; the library works on its
        # own stream and synchronises it before returning, so the current
        # stream is drained first and the two never overlap on them
        torch = self._torch
        di = torch.as_tensor(np.ascontiguousarray(idx, dtype=np.int32)).to(self.device)
        out = torch.empty((di.numel(), width), dtype=torch.float32, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        self._check(fn(self.h, C.c_void_p(di.data_ptr()), int(di.numel()), C.c_void_p(out.data_ptr())),
                    self.h)
        return out

    def factor_features(self, idx) -> "torch.Tensor":
        """Features (n x 16, device) of factors idx (caller order); advances
        the feature history."""
        return self._device_rows(self._lib.gbp_factor_features, idx, _capi.MLP_FEATURES)

    def factor_messages(self, idx) -> "torch.Tensor":
        """Message rows (n x 16, device) of factors idx (caller order)."""
        return self._device_rows(self._lib.gbp_factor_messages, idx, 16)


# ----------------------------------------------------------------------------
# learned damping network (stateless C entry points on caller device buffers)
# ----------------------------------------------------------------------------

def _check_plain(st):
    if st != 0:
        raise GBPError(st, _capi.load().gbp_last_error(None).decode())


def mlp_infer(weights_bf16, x, stream=None):
    """Damping and log-depth heads of the network for feature rows x
    (n x 16 CUDA tensor, float32, or bfloat16 for gbp_mlp_infer_bf16);
    weights_bf16 is a CUDA tensor holding the BF16 bit patterns (int16 or
    uint16, MLP_PARAMS entries)."""
    import torch
    lib = _capi.load()
    if x.dtype not in (torch.float32, torch.bfloat16) or not x.is_cuda or x.dim() != 2 or x.shape[1] != MLP_FEATURES:
        raise ValueError("x must be a CUDA float32 or bfloat16 tensor of shape (n, 16)")
    if weights_bf16.numel() != MLP_PARAMS or weights_bf16.element_size() != 2 or not weights_bf16.is_cuda:
        raise ValueError("weights must be a CUDA tensor of MLP_PARAMS 16-bit values")
    x = x.contiguous()
    weights_bf16 = weights_bf16.contiguous()
    n = x.shape[0]
    d = torch.empty(n, dtype=torch.float32, device=x.device)
    delta = torch.empty(n, dtype=torch.float32, device=x.device)
    s = stream if stream is not None else torch.cuda.current_stream(x.device)
    fn = lib.gbp_mlp_infer if x.dtype == torch.float32 else lib.gbp_mlp_infer_bf16
    _check_plain(fn(C.c_void_p(weights_bf16.data_ptr()), C.c_void_p(x.data_ptr()), n,
                    C.c_void_p(d.data_ptr()), C.c_void_p(delta.data_ptr()), C.c_void_p(s.cuda_stream)))
    return d, delta


def init_mlp_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights and zero biases in the parameter-blob layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for rows, cols in ((64, 16), (64, 64), (2, 64)):
        lim = np.sqrt(6.0 / cols)
        parts.append(rng.uniform(-lim, lim, rows * cols))
        parts.append(np.zeros(rows))
    return np.concatenate(parts).astype(np.float32)


def bf16_bits(theta) -> np.ndarray:
    """Round-to-nearest-even BF16 bit patterns of float32 values."""
    u = np.ascontiguousarray(theta, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)


class MLPTrainer:
    """FP32 master weights, Adam moments and the BF16 copy of the network on
    the GPU; each step calls gbp_mlp_train_step on a batch of rows of the
    data set held on the device."""

    def __init__(self, theta0=None, *, max_batch: int = 8192, seed: int = 0, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("MLPTrainer needs a ROCm GPU")
        self._lib = _capi.load()
        self.device = torch.device("cuda", device)
        th = init_mlp_params(seed) if theta0 is None else np.asarray(theta0, dtype=np.float32)
        if th.shape != (MLP_PARAMS,):
            raise ValueError(f"theta must have {MLP_PARAMS} entries")
        self.theta = torch.as_tensor(th.copy()).to(self.device)
        self.m = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=self.device)
        self.v = torch.zeros_like(self.m)
        self.grad = torch.zeros_like(self.m)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.w = torch.as_tensor(bf16_bits(th).view(np.int16).copy()).to(self.device)
        nbytes = C.c_size_t(0)
        _check_plain(self._lib.gbp_mlp_train_workspace_bytes(int(max_batch), C.byref(nbytes)))
        self.max_batch = int(max_batch)
        self.ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.steps = 0
        self.x = self.y = self.mask = None

    def set_data(self, x, y, mask) -> None:
        import torch
        self.x = torch.as_tensor(x, dtype=torch.float32).to(self.device).contiguous()
        self.y = torch.as_tensor(y, dtype=torch.float32).to(self.device).contiguous()
        self.mask = torch.as_tensor(mask, dtype=torch.float32).to(self.device).contiguous()
        if self.x.shape[1:] != (MLP_FEATURES,) or self.y.shape != (self.x.shape[0], 2) or \
                self.mask.shape != self.y.shape:
            raise ValueError("data shapes must be (n, 16), (n, 2), (n, 2)")

    def _call(self, idx, lr, step):
        import torch
        if self.x is None:
            raise RuntimeError("set_data first")
        idx = torch.as_tensor(idx, dtype=torch.int32).to(self.device).contiguous()
        if not 1 <= idx.numel() <= self.max_batch:
            raise ValueError("batch size must be in [1, max_batch]")
        s = torch.cuda.current_stream(self.device)
        P = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
        _check_plain(self._lib.gbp_mlp_train_step(
            P(self.x), P(self.y), P(self.mask), int(self.x.shape[0]), P(idx), int(idx.numel()),
            P(self.theta), P(self.m), P(self.v), P(self.w), float(lr), int(step), P(self.grad),
            P(self.loss), P(self.ws), self.ws.numel(), C.c_void_p(s.cuda_stream)))
        self._last_idx = idx  # keep the index buffer alive until the stream has used it

    def step(self, idx, lr: float = 1e-3):
        """One Adam step on rows idx; returns the batch loss tensor (device)."""
        self.steps += 1
        self._call(idx, lr, self.steps)
        return self.loss

    def gradient(self, idx):
        """(gradient, loss) on rows idx without updating anything."""
        self._call(idx, 0.0, 0)
        return self.grad.clone(), float(self.loss.item())

    def theta_host(self) -> np.ndarray:
        return self.theta.cpu().numpy().astype(np.float32)

    def weights_bf16(self) -> np.ndarray:
        """BF16 bit patterns of the current master weights."""
        return self.w.cpu().numpy().view(np.uint16).copy()
