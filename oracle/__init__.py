"""FP64 CPU oracle for synchronous GBP bundle adjustment.

TEST INFRASTRUCTURE: this package is the reference the HIP library is
checked against. Only the test suite, the smoke check and the benchmark's
CPU-baseline leg import it. It shares no code with the HIP library.

The arithmetic lives in `gbp_oracle.c` (plain C, FP64, IEEE round-to-nearest,
no fast-math), compiled into `liboracle.so` by `oracle.build`. This module only
marshals arguments.
"""
from __future__ import annotations

import ctypes as C
import os
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_up = C.POINTER(C.c_ubyte)


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from .build import build
            build()
        lib = C.CDLL(path)
        lib.oracle_create.restype = C.c_void_p
        lib.oracle_create.argtypes = [C.c_int, C.c_int, C.c_int, _ip, _ip, _dp, _dp,
                                      _dp, _dp, _dp, _dp]
        lib.oracle_destroy.argtypes = [C.c_void_p]
        lib.oracle_relinearise.argtypes = [C.c_void_p, C.c_double]
        lib.oracle_relinearise.restype = C.c_int
        lib.oracle_iterate.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double]
        lib.oracle_iterate.restype = C.c_int
        lib.oracle_beliefs.argtypes = [C.c_void_p] + [_dp] * 6
        lib.oracle_reproj.argtypes = [C.c_void_p, _dp, _dp, _up]
        lib.oracle_factor.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp]
        lib.oracle_prior.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp]
        lib.oracle_messages.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        lib.oracle_time.argtypes = [C.c_void_p]
        lib.oracle_time.restype = C.c_int
        lib.oracle_counters.argtypes = [C.c_void_p, _ip, _up]
        lib.oracle_add.argtypes = [C.c_void_p, C.c_int, _dp, _dp, C.c_int, _dp,
                                   C.c_int, _ip, _ip, _dp]
        lib.oracle_add.restype = C.c_int
        lib.oracle_project.argtypes = [_dp, _dp, _dp, _dp, _dp]
        lib.oracle_project.restype = C.c_double
        lib.oracle_so3_exp.argtypes = [_dp, _dp]
        lib.oracle_so3_jr.argtypes = [_dp, _dp]
        lib.oracle_huber_weight.argtypes = [C.c_double, C.c_double]
        lib.oracle_huber_weight.restype = C.c_double
        lib.oracle_threads.restype = C.c_int
        lib.oracle_set_threads.argtypes = [C.c_int]
        lib.oracle_odometry.argtypes = [_dp, _dp, _dp, _dp]
        lib.oracle_add_pairs.argtypes = [C.c_void_p, C.c_int, C.c_int, _ip, _ip, _dp, _dp]
        lib.oracle_add_pairs.restype = C.c_int
        lib.oracle_pair_messages.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp]
        _LIB = lib
    return _LIB


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


def _out(shape):
    a = np.zeros(shape, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def project(x, l, cam):
    """h(x, l), its 2x9 Jacobian and the camera depth (cam = fx, fy, cx, cy)."""
    x, px = _d(x)
    l, pl = _d(l)
    c, pc = _d(np.asarray(cam, dtype=np.float64)[:4])
    h, ph = _out(2)
    J, pJ = _out((2, 9))
    pz = _lib().oracle_project(px, pl, pc, ph, pJ)
    return h, J, pz


def so3_exp(w):
    w, pw = _d(w)
    R, pR = _out((3, 3))
    _lib().oracle_so3_exp(pw, pR)
    return R


def so3_jr(w):
    w, pw = _d(w)
    R, pR = _out((3, 3))
    _lib().oracle_so3_jr(pw, pR)
    return R


def huber_weight(M, N):
    return _lib().oracle_huber_weight(float(M), float(N))


def threads() -> int:
    return _lib().oracle_threads()


def odometry(xa, xb):
    """Odometry measurement c_b - c_a (camera centres c = -R(omega)^T t) and
    its 3x12 Jacobian w.r.t. [x_a; x_b]."""
    a, pa = _d(np.asarray(xa, dtype=np.float64).reshape(6))
    b, pb = _d(np.asarray(xb, dtype=np.float64).reshape(6))
    h, ph = _out(3)
    J, pJ = _out((3, 12))
    _lib().oracle_odometry(pa, pb, ph, pJ)
    return h, J


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's loops (results do not depend on it)."""
    _lib().oracle_set_threads(int(n))


class Oracle:
    """One BA problem under the oracle. Hyperparameter defaults are the
    paper's (Section 8): beta 0.01, relinearise at most every 10 iterations,
    undamped for 8 iterations after relinearising, priors weakened to 1/100
    (annealed over 10 iterations when `anneal` is set). Damping acts on the
    eta message only unless `damp_lambda` is set."""

    def __init__(self, problem, *, beta=0.01, relin_interval=10, undamped=8,
                 anneal_iters=10, weaken=0.01, anneal=False, huber_k=2.0,
                 zmin=1e-3, damp_lambda=False, kf_init=None, lm_init=None):
        lib = _lib()
        p = problem
        self.problem = p
        self.nk, self.nl, self.nf = p.n_keyframes, p.n_landmarks, p.n_factors
        self._keep = []
        fkf, pfkf = _i(p.factor_kf)
        flm, pflm = _i(p.factor_lm)
        kfi, pkfi = _d(p.kf_init if kf_init is None else kf_init)
        lmi, plmi = _d(p.lm_init if lm_init is None else lm_init)
        anc, panc = _d(p.kf_anchor_info)
        z, pz = _d(p.z)
        cam, pcam = _d(np.array([p.cam.fx, p.cam.fy, p.cam.cx, p.cam.cy,
                                 p.cam.sigma, zmin]))
        opt, popt = _d(np.array([beta, relin_interval, undamped, anneal_iters,
                                 weaken, 1.0 if anneal else 0.0, huber_k,
                                 1.0 if damp_lambda else 0.0]))
        self.h = lib.oracle_create(self.nk, self.nl, self.nf, pfkf, pflm, pkfi,
                                   plmi, panc, pz, pcam, popt)
        if not self.h:
            raise MemoryError("oracle_create failed")
        self.huber_k = huber_k
        self.sigma = p.cam.sigma
        self._cur_z = np.array(p.z, dtype=np.float64)

    def __del__(self):
        if getattr(self, "h", None):
            _lib().oracle_destroy(self.h)
            self.h = None

    @property
    def t(self) -> int:
        return _lib().oracle_time(self.h)

    def relinearise(self, beta: float = -1.0) -> int:
        return _lib().oracle_relinearise(self.h, float(beta))

    def iterate(self, n: int, damping: float = 0.4, huber_k=None) -> None:
        if huber_k is not None:
            self.huber_k = huber_k
        rc = _lib().oracle_iterate(self.h, int(n), float(damping), float(self.huber_k))
        if rc != 0:
            raise FloatingPointError("oracle: singular system during iteration")

    def beliefs(self) -> dict:
        kf_mu, a = _out((self.nk, 6))
        lm_mu, b = _out((self.nl, 3))
        kf_lam, c = _out((self.nk, 6, 6))
        lm_lam, d = _out((self.nl, 3, 3))
        kf_eta, e = _out((self.nk, 6))
        lm_eta, f = _out((self.nl, 3))
        _lib().oracle_beliefs(self.h, a, b, c, d, e, f)
        return dict(kf_mu=kf_mu, lm_mu=lm_mu, kf_lam=kf_lam, lm_lam=lm_lam,
                    kf_eta=kf_eta, lm_eta=lm_eta)

    def reproj(self, zref=None, mask=None) -> dict:
        out, po = _out(9)
        if zref is not None:
            zr, pzr = _d(zref)
            mk = np.ascontiguousarray(mask, dtype=np.uint8)
            _lib().oracle_reproj(self.h, po, pzr, mk.ctypes.data_as(_up))
        else:
            _lib().oracle_reproj(self.h, po, None, None)
        return dict(are_all=out[0], are_quadratic=out[1], n_valid=int(out[2]),
                    n_quadratic=int(out[3]), n_linear=int(out[4]),
                    n_invalid=int(out[5]), are_ref=out[6], n_ref=int(out[7]),
                    n_linear_ref=int(out[8]))

    def factor(self, f: int):
        eta, a = _out(9)
        lam, b = _out((9, 9))
        lin, c = _out(9)
        w, d = _out(1)
        _lib().oracle_factor(self.h, int(f), a, b, c, d)
        return eta, lam, lin, float(w[0])

    def prior(self, t: int):
        kd, a = _out((self.nk, 6))
        ke, b = _out((self.nk, 6))
        ld, c = _out((self.nl, 3))
        le, d = _out((self.nl, 3))
        _lib().oracle_prior(self.h, int(t), a, b, c, d)
        return kd, ke, ld, le

    def messages(self) -> dict:
        ke, a = _out((self.nf, 6))
        kl, b = _out((self.nf, 6, 6))
        le, c = _out((self.nf, 3))
        ll, d = _out((self.nf, 3, 3))
        _lib().oracle_messages(self.h, a, b, c, d)
        return dict(k_eta=ke, k_lam=kl, l_eta=le, l_lam=ll)

    def counters(self):
        cnt = np.zeros(self.nf, dtype=np.int32)
        inv = np.zeros(self.nf, dtype=np.uint8)
        _lib().oracle_counters(self.h, cnt.ctypes.data_as(_ip), inv.ctypes.data_as(_up))
        return cnt, inv

    def add_pairs(self, kind: int, a, b, z, prec) -> None:
        """Pairwise factors: kind 0, keyframe difference x_b - x_a ~ N(z,
        diag(prec)^-1) (6 values); kind 1, the same between landmarks (3);
        kind 2, keyframe odometry c_b - c_a ~ N(z, diag(prec)^-1) (3)."""
        D = 6 if kind == 0 else 3
        a_, pa = _i(np.asarray(a).ravel())
        b_, pb = _i(np.asarray(b).ravel())
        z_, pz = _d(np.asarray(z, dtype=np.float64).reshape(-1, D))
        p_, pp = _d(np.asarray(prec, dtype=np.float64).reshape(-1, D))
        if not (len(a_) == len(b_) == len(z_) == len(p_)):
            raise ValueError("a, b, z and prec need one entry per factor")
        self._keep += [a_, b_, z_, p_]
        if _lib().oracle_add_pairs(self.h, int(kind), len(a_), pa, pb, pz, pp) != 0:
            raise ValueError("oracle_add_pairs rejected the factors")
        self.n_pairs = getattr(self, "n_pairs", [0, 0, 0])
        self.n_pairs[kind] += len(a_)

    def pair_messages(self, kind: int) -> dict:
        D = 3 if kind == 1 else 6
        n = getattr(self, "n_pairs", [0, 0, 0])[kind]
        ae, pa = _out((n, D))
        al, pb = _out((n, D, D))
        be, pc = _out((n, D))
        bl, pd = _out((n, D, D))
        _lib().oracle_pair_messages(self.h, int(kind), pa, pb, pc, pd)
        return dict(a_eta=ae, a_lam=al, b_eta=be, b_lam=bl)

    def add(self, kf_init, lm_init, f_kf, f_lm, z, kf_anchor_info=None) -> None:
        kf_init = np.atleast_2d(np.asarray(kf_init, dtype=np.float64)).reshape(-1, 6)
        lm_init = np.asarray(lm_init, dtype=np.float64).reshape(-1, 3)
        nkn, nln = kf_init.shape[0], lm_init.shape[0]
        a, pa = _d(kf_init)
        anc = np.zeros(nkn) if kf_anchor_info is None else kf_anchor_info
        an, pan = _d(anc)
        b, pb = _d(lm_init)
        fk, pfk = _i(f_kf)
        fl, pfl = _i(f_lm)
        zz, pzz = _d(np.asarray(z).reshape(-1, 2))
        rc = _lib().oracle_add(self.h, nkn, pa, pan, nln, pb, len(fk), pfk, pfl, pzz)
        if rc != 0:
            raise ValueError("oracle_add: bad indices")
        self.nk += nkn
        self.nl += nln
        self.nf += len(fk)
