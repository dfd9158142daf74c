"""ctypes wrapper of the FP64 LEAD oracle (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this module.  It loads ``oracle/liblead_oracle.so`` built by
``oracle/build.py`` with gcc; it never touches the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LEAD_ORACLE_LIB", os.path.join(HERE, "liblead_oracle.so"))

Z, X = 0, 1
MINSUM, SUMPRODUCT = 0, 1
FULL, LOCAL = 0, 1


class Params(C.Structure):
    _fields_ = [("alpha", C.c_double), ("bp", C.c_int), ("ms_scale", C.c_double),
                ("max_iter_local", C.c_int), ("max_iter_global", C.c_int),
                ("llr_clamp", C.c_double), ("early_exit", C.c_int), ("stage", C.c_int),
                ("boost", C.c_int), ("perturb", C.c_double), ("perturb_seed", C.c_uint64),
                ("local_osd", C.c_int), ("global_osd", C.c_int), ("osd_order", C.c_int),
                ("osd_exact", C.c_int)]


def params(alpha=1.0, bp=MINSUM, ms_scale=0.75, max_iter_local=32, max_iter_global=32,
           llr_clamp=30.0, early_exit=1, stage=FULL, boost=1, perturb=0.0, perturb_seed=0,
           local_osd=0, global_osd=0, osd_order=0, osd_exact=0) -> Params:
    return Params(alpha, bp, ms_scale, max_iter_local, max_iter_global, llr_clamp,
                  early_exit, stage, boost, perturb, perturb_seed, local_osd, global_osd, osd_order,
                  osd_exact)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.oracle_build.restype = C.c_int
        L.oracle_build.argtypes = [C.c_int, P, C.c_int, P, P, C.c_int, P, C.c_int, P,
                                   C.POINTER(C.c_void_p), C.c_char_p, C.c_int]
        L.oracle_free.argtypes = [C.c_void_p]
        L.oracle_info.argtypes = [C.c_void_p, P]
        L.oracle_views.argtypes = [C.c_void_p, C.c_int, P]
        L.oracle_hloc.argtypes = [C.c_void_p, C.c_int, P]
        L.oracle_H.argtypes = [C.c_void_p, C.c_int, P]
        L.oracle_logicals.argtypes = [C.c_void_p, C.c_int, P]
        L.oracle_syndrome.argtypes = [C.c_void_p, C.c_int, C.c_int, P, C.c_int, P, C.c_int]
        L.oracle_decode.restype = C.c_int
        L.oracle_decode.argtypes = [C.c_void_p, C.c_int, C.POINTER(Params), C.c_int, P, C.c_int,
                                    P, P, C.c_int, P, P, P, P, P]
        L.oracle_aggregate.argtypes = [C.c_int, C.c_int, C.c_int, P, P, C.c_double, C.c_double,
                                       P, P]
        L.oracle_bp.restype = C.c_int
        L.oracle_bp.argtypes = [C.c_int, C.c_int, P, P, P, C.POINTER(Params), C.c_int, P, P,
                                C.POINTER(C.c_int)]
        L.oracle_global_bp.restype = C.c_int
        L.oracle_osd0.restype = C.c_int
        L.oracle_osd0.argtypes = [C.c_int, C.c_int, P, P, P, P]
        L.oracle_osd.restype = C.c_int
        L.oracle_osd.argtypes = [C.c_int, C.c_int, P, P, P, P, C.c_int, P]
        L.oracle_osd_ex.restype = C.c_int
        L.oracle_osd_ex.argtypes = [C.c_int, C.c_int, P, P, P, P, C.c_int, C.c_int, P]
        L.oracle_osd_weight.restype = C.c_long
        L.oracle_osd_weight.argtypes = [C.c_double]
        L.oracle_global_bp.argtypes = [C.c_void_p, C.c_int, C.POINTER(Params), C.c_int, P,
                                       C.c_int, P, P, C.c_int, P, P]
        L.oracle_logical_failure.restype = C.c_int
        L.oracle_logical_failure.argtypes = [C.c_void_p, C.c_int, P, C.c_int]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


@dataclass
class Info:
    order: int
    delta: int
    n: int
    r: tuple
    m: tuple
    rank: tuple
    k: int
    eloc: tuple


class OracleCode:
    """The code built by the oracle from (G, A, B, C_A, C_B)."""

    def __init__(self, mul, delta, A, B, GA, GB):
        L = lib()
        mul = np.ascontiguousarray(mul, dtype=np.uint16)
        order = mul.shape[0]
        A = np.ascontiguousarray(A, dtype=np.int32)
        B = np.ascontiguousarray(B, dtype=np.int32)
        GA = np.ascontiguousarray([int(x) for x in GA], dtype=np.uint64)
        GB = np.ascontiguousarray([int(x) for x in GB], dtype=np.uint64)
        h = C.c_void_p()
        err = C.create_string_buffer(512)
        rc = L.oracle_build(order, _p(mul), delta, _p(A), _p(B), len(GA), _p(GA), len(GB), _p(GB),
                            C.byref(h), err, 512)
        if rc != 0:
            raise OracleError(rc, err.value.decode())
        self._h = h
        info = np.zeros(12, dtype=np.int32)
        L.oracle_info(h, _p(info))
        self.info = Info(int(info[0]), int(info[1]), int(info[2]), (int(info[3]), int(info[4])),
                         (int(info[5]), int(info[6])), (int(info[7]), int(info[8])), int(info[9]),
                         (int(info[10]), int(info[11])))

    @classmethod
    def from_spec(cls, spec):
        return cls(spec.mul, spec.delta, spec.A, spec.B, spec.GA, spec.GB)

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().oracle_free(self._h)
                self._h = None
        except Exception:
            pass

    @property
    def n(self):
        return self.info.n

    @property
    def k(self):
        return self.info.k

    def m(self, t=Z):
        return self.info.m[t]

    def views(self, t=Z) -> np.ndarray:
        d2 = self.info.delta ** 2
        out = np.zeros((self.info.order, d2), dtype=np.int32)
        lib().oracle_views(self._h, t, _p(out))
        return out

    def hloc(self, t=Z) -> np.ndarray:
        out = np.zeros((self.info.r[t], self.info.delta ** 2), dtype=np.uint8)
        lib().oracle_hloc(self._h, t, _p(out))
        return out

    def H(self, t=Z) -> np.ndarray:
        out = np.zeros((self.info.m[t], self.info.n), dtype=np.uint8)
        lib().oracle_H(self._h, t, _p(out))
        return out

    def logicals(self, t=Z) -> np.ndarray:
        out = np.zeros((self.info.k, self.info.n), dtype=np.uint8)
        lib().oracle_logicals(self._h, t, _p(out))
        return out

    def syndrome(self, err_packed: np.ndarray, t=Z) -> np.ndarray:
        err_packed = np.ascontiguousarray(err_packed, dtype=np.uint64)
        shots, ew = err_packed.shape
        sw = (self.info.m[t] + 63) // 64
        out = np.zeros((shots, sw), dtype=np.uint64)
        lib().oracle_syndrome(self._h, t, shots, _p(err_packed), ew, _p(out), sw)
        return out

    def _prior(self, prior, shots):
        prior = np.asarray(prior, dtype=np.float64)
        n = self.info.n
        if prior.ndim == 0:
            prior = np.full((shots, n), float(prior))
        elif prior.ndim == 1 and prior.shape[0] == shots and shots != n:
            prior = np.repeat(prior[:, None], n, axis=1)
        elif prior.ndim == 1:
            prior = np.broadcast_to(prior, (shots, n))
        return np.ascontiguousarray(prior, dtype=np.float64)

    def decode(self, synd: np.ndarray, prior, t=Z, p: Params = None, want_local=False):
        """LEAD decode.  `prior`: scalar, per-shot [S], shared [n] or full
        [S, n] channel LLRs (float32 values are promoted exactly)."""
        p = p or params()
        synd = np.ascontiguousarray(synd, dtype=np.uint64)
        shots, sw = synd.shape
        n = self.info.n
        prior = self._prior(prior, shots)
        ew = (n + 63) // 64
        ehat = np.zeros((shots, ew), dtype=np.uint64)
        post = np.zeros((shots, n), dtype=np.float64)
        lam = np.zeros((shots, n), dtype=np.float64)
        stats = np.zeros((shots, 6), dtype=np.int32)
        margin = np.zeros(shots, dtype=np.float64)
        loc = (np.zeros((shots, self.info.order, self.info.delta ** 2), dtype=np.float64)
               if want_local else None)
        rc = lib().oracle_decode(self._h, t, C.byref(p), shots, _p(synd), sw, _p(prior), _p(ehat), ew,
                                 _p(post), _p(lam), _p(stats), _p(margin), _p(loc))
        if rc != 0:
            raise OracleError(rc, "oracle_decode failed")
        out = dict(ehat=ehat, post=post, lam=lam, stats=np.ascontiguousarray(stats[:, :5]), osd_views=stats[:, 5].copy(),
                   margin=margin)
        if want_local:
            out["local"] = loc
        return out

    def global_bp(self, synd, prior, t=Z, p: Params = None):
        p = p or params()
        synd = np.ascontiguousarray(synd, dtype=np.uint64)
        shots, sw = synd.shape
        n = self.info.n
        prior = self._prior(prior, shots)
        ew = (n + 63) // 64
        ehat = np.zeros((shots, ew), dtype=np.uint64)
        post = np.zeros((shots, n), dtype=np.float64)
        stats = np.zeros((shots, 2), dtype=np.int32)
        lib().oracle_global_bp(self._h, t, C.byref(p), shots, _p(synd), sw, _p(prior), _p(ehat), ew,
                               _p(post), _p(stats))
        return dict(ehat=ehat, post=post, stats=stats)

    def logical_failure(self, residual_packed: np.ndarray, t=Z, route=0) -> np.ndarray:
        residual_packed = np.ascontiguousarray(residual_packed, dtype=np.uint64)
        if residual_packed.ndim == 1:
            residual_packed = residual_packed[None]
        out = np.zeros(residual_packed.shape[0], dtype=bool)
        for i in range(residual_packed.shape[0]):
            row = np.ascontiguousarray(residual_packed[i])
            out[i] = bool(lib().oracle_logical_failure(self._h, t, _p(row), route))
        return out


def aggregate(n: int, view: np.ndarray, pv: np.ndarray, alpha: float, llr_clamp: float = 30.0):
    """Phase 2 alone.  view, pv: [nviews, vsize].  Returns (phat, lambda')."""
    view = np.ascontiguousarray(view, dtype=np.int32)
    pv = np.ascontiguousarray(pv, dtype=np.float64)
    nv, vs = view.shape
    phat = np.zeros(n, dtype=np.float64)
    lam = np.zeros(n, dtype=np.float64)
    lib().oracle_aggregate(n, nv, vs, _p(view), _p(pv), alpha, llr_clamp, _p(phat), _p(lam))
    return phat, lam


def bp(H: np.ndarray, s: np.ndarray, lam: np.ndarray, max_iter: int, p: Params = None):
    """Plain BP on a dense 0/1 matrix.  Returns (L, e, conv, iterations)."""
    p = p or params()
    H = np.ascontiguousarray(H, dtype=np.uint8)
    rows, cols = H.shape
    s = np.ascontiguousarray(s, dtype=np.uint8)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    L = np.zeros(cols, dtype=np.float64)
    e = np.zeros(cols, dtype=np.uint8)
    conv = C.c_int(0)
    it = lib().oracle_bp(rows, cols, _p(H), _p(s), _p(lam), C.byref(p), max_iter, _p(L), _p(e),
                         C.byref(conv))
    return L, e, bool(conv.value), it


def osd0(H: np.ndarray, s: np.ndarray, L: np.ndarray):
    """OSD-0 of H e = s with reliabilities L (most likely in error first:
    round(64 L) ascending, ties in position order).  Returns (e, ok)."""
    H = np.ascontiguousarray(H, dtype=np.uint8)
    s = np.ascontiguousarray(s, dtype=np.uint8)
    L = np.ascontiguousarray(L, dtype=np.float64)
    rows, cols = H.shape
    e = np.zeros(cols, dtype=np.uint8)
    rc = lib().oracle_osd0(rows, cols, _p(H), _p(s), _p(L), _p(e))
    return e, rc == 0


def osd(H: np.ndarray, s: np.ndarray, L: np.ndarray, prior=None, order: int = 0, exact: bool = False):
    """OSD of H e = s: ranking by round(64 L) as osd0; order >= 1 adds the
    combination sweep with costs from the prior LLRs.  exact: rank by L and
    price in FP64 instead.  Returns (e, ok)."""
    H = np.ascontiguousarray(H, dtype=np.uint8)
    s = np.ascontiguousarray(s, dtype=np.uint8)
    L = np.ascontiguousarray(L, dtype=np.float64)
    rows, cols = H.shape
    pr = np.ascontiguousarray(np.zeros(cols) if prior is None else prior, dtype=np.float64)
    e = np.zeros(cols, dtype=np.uint8)
    rc = lib().oracle_osd_ex(rows, cols, _p(H), _p(s), _p(L), _p(pr), int(order), int(exact), _p(e))
    return e, rc == 0


def osd_weight(lam: float) -> int:
    """Cost of setting a bit with prior LLR lam in the combination sweep."""
    return int(lib().oracle_osd_weight(float(lam)))
