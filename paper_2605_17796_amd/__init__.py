"""LEAD decoding of quantum Tanner codes on MI355X.

Thin binding over the C ABI of ``liblead.so`` (declared in include/lead.h).
Every step of decoding runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch provides device memory and streams.

Low-level functions carry the C names (``lead_code_create``,
``lead_decode`` ...).  ``Code`` and ``Decoder`` wrap them for torch tensors.
Loading fails loudly if the library has not been built
(``python -m paper_2605_17796_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblead.so")

LEAD_OK = 0
LEAD_CHECK_Z, LEAD_CHECK_X = 0, 1
LEAD_PRIOR_PER_SHOT, LEAD_PRIOR_SHARED, LEAD_PRIOR_FULL = 0, 1, 2
LEAD_STAGE_FULL, LEAD_STAGE_LOCAL, LEAD_STAGE_GLOBAL = 0, 1, 2
LEAD_BP_MINSUM, LEAD_BP_SUMPRODUCT = 0, 1
STATUS_NAMES = {0: "LEAD_OK", -1: "LEAD_E_ARG", -2: "LEAD_E_GROUP", -3: "LEAD_E_SYMMETRY", -4: "LEAD_E_TNC",
                -5: "LEAD_E_LOCALCODE", -6: "LEAD_E_NOMEM", -7: "LEAD_E_DEVICE", -8: "LEAD_E_CAPACITY",
                -9: "LEAD_E_UNSUPPORTED", -10: "LEAD_E_CLOSED"}


class LeadError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class lead_code_desc(C.Structure):
    _fields_ = [("order", C.c_int32), ("mul", C.c_void_p), ("delta", C.c_int32), ("A", C.c_void_p),
                ("B", C.c_void_p), ("kA", C.c_int32), ("kB", C.c_int32), ("GA", C.c_void_p),
                ("GB", C.c_void_p)]


class lead_code_info(C.Structure):
    _fields_ = [("order", C.c_int32), ("delta", C.c_int32), ("n", C.c_int32), ("r", C.c_int32 * 2),
                ("m", C.c_int32 * 2), ("rank", C.c_int32 * 2), ("k", C.c_int32), ("eloc", C.c_int32 * 2)]


class lead_params(C.Structure):
    _fields_ = [("alpha", C.c_float), ("ms_scale", C.c_float), ("max_iter_local", C.c_int32),
                ("max_iter_global", C.c_int32), ("llr_clamp", C.c_float), ("early_exit", C.c_int32),
                ("stage", C.c_int32), ("boost", C.c_int32), ("fixed_point_stop", C.c_int32), ("local_post", C.c_int32),
                ("bp", C.c_int32), ("global_post", C.c_int32), ("osd_order", C.c_int32)]


class lead_schedule(C.Structure):
    _fields_ = [("shots_per_workgroup", C.c_int32), ("fused", C.c_int32), ("local_chunk", C.c_int32),
                ("local_waves", C.c_int32), ("specialized", C.c_int32), ("chunk_shots", C.c_int32),
                ("global_osd_form", C.c_int32), ("global_tiles", C.c_int32)]


class lead_phase_times(C.Structure):
    _fields_ = [("local_ms", C.c_double), ("global_ms", C.c_double), ("local_launches", C.c_int64),
                ("global_launches", C.c_int64)]


class lead_batch_item(C.Structure):
    _fields_ = [("decoder", C.c_void_p), ("shots", C.c_int64), ("d_synd", C.c_void_p), ("synd_words", C.c_int64),
                ("d_prior", C.c_void_p), ("mode", C.c_int32), ("d_ehat", C.c_void_p), ("ehat_words", C.c_int64),
                ("d_post", C.c_void_p), ("d_prior_llr", C.c_void_p), ("d_stats", C.c_void_p)]


class lead_server_config(C.Structure):
    _fields_ = [("mem_budget_bytes", C.c_int64), ("max_batch_shots", C.c_int32),
                ("max_slots_per_decoder", C.c_int32), ("return_posteriors", C.c_int32), ("reserved", C.c_int32),
                ("max_pending_shots", C.c_int64)]


class lead_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("shots_completed", C.c_int64),
                ("launches", C.c_int64), ("slots", C.c_int32), ("slots_created", C.c_int32),
                ("slot_bytes", C.c_int64), ("evictions", C.c_int64), ("refused", C.c_int64),
                ("pending_shots", C.c_int64)]


STATS_FIELDS = ("converged", "global_iters", "local_iters_sum", "local_iters_max", "local_converged_views",
                "local_fixed_views", "global_fixed_iter", "local_osd_views")

SYMBOLS = ["lead_last_error", "lead_code_create", "lead_code_query", "lead_code_get_H", "lead_code_get_views",
           "lead_code_specialize", "lead_code_destroy", "lead_decoder_create", "lead_decoder_set_params", "lead_decoder_destroy",
           "lead_decode", "lead_decode_noalloc", "lead_decode_plain", "lead_syndrome", "lead_decoder_set_schedule",
           "lead_decoder_get_schedule", "lead_decoder_time_phases", "lead_decoder_phase_times",
           "lead_decoder_autotune", "lead_batch_decode", "lead_batch_graph_create",
           "lead_batch_graph_launch", "lead_batch_graph_destroy", "lead_batch_fused_create", "lead_batch_fused_launch",
           "lead_batch_fused_destroy", "lead_batch_fused_specialize", "lead_server_create", "lead_server_submit",
           "lead_server_poll", "lead_server_wait", "lead_server_result", "lead_server_get_stats",
           "lead_server_clock_ns", "lead_server_close", "lead_server_destroy"]

_lib = None


def lib():
    """The loaded liblead.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_17796_amd.build`")
        # torch ships its own HIP runtime (soname libamdhip64.so.7).  Loading it
        # first makes liblead.so bind to that same runtime instead of pulling a
        # second copy from /opt/rocm into the process.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        L.lead_last_error.restype = C.c_char_p
        L.lead_code_create.argtypes = [C.POINTER(lead_code_desc), C.POINTER(P)]
        L.lead_code_query.argtypes = [P, C.POINTER(lead_code_info)]
        L.lead_code_get_H.argtypes = [P, I32, P, P]
        L.lead_code_get_views.argtypes = [P, I32, P]
        L.lead_code_specialize.argtypes = [P, I32]
        L.lead_code_destroy.argtypes = [P]
        L.lead_code_destroy.restype = None
        L.lead_decoder_create.argtypes = [P, I32, C.POINTER(lead_params), I64, C.POINTER(P)]
        L.lead_decoder_set_params.argtypes = [P, C.POINTER(lead_params)]
        L.lead_decoder_set_schedule.argtypes = [P, C.POINTER(lead_schedule)]
        L.lead_decoder_get_schedule.argtypes = [P, C.POINTER(lead_schedule)]
        L.lead_decoder_time_phases.argtypes = [P, I32]
        L.lead_decoder_phase_times.argtypes = [P, C.POINTER(lead_phase_times)]
        L.lead_decoder_destroy.argtypes = [P]
        L.lead_decoder_destroy.restype = None
        dec_args = [P, I64, P, I64, P, I32, P, I64, P, P, P, P]
        L.lead_decode.argtypes = dec_args
        L.lead_decode_noalloc.argtypes = dec_args
        L.lead_decode_plain.argtypes = dec_args
        L.lead_syndrome.argtypes = [P, I64, P, I64, P, I64, P]
        L.lead_decoder_autotune.argtypes = [P, I64, P, I64, P, I32, P, C.POINTER(lead_schedule)]
        L.lead_batch_decode.argtypes = [C.POINTER(lead_batch_item), I32, P]
        L.lead_batch_graph_create.argtypes = [C.POINTER(lead_batch_item), I32, P, C.POINTER(P)]
        L.lead_batch_graph_launch.argtypes = [P, P]
        L.lead_batch_graph_destroy.argtypes = [P]
        L.lead_batch_graph_destroy.restype = None
        L.lead_batch_fused_create.argtypes = [C.POINTER(lead_batch_item), I32, C.POINTER(P)]
        L.lead_batch_fused_launch.argtypes = [P, P]
        L.lead_batch_fused_destroy.argtypes = [P]
        L.lead_batch_fused_destroy.restype = None
        L.lead_batch_fused_specialize.argtypes = [P, P, P, P, I32]
        L.lead_server_create.argtypes = [C.POINTER(P), I32, C.POINTER(lead_server_config), C.POINTER(P)]
        L.lead_server_submit.argtypes = [P, I32, I64, P, I64, P, C.POINTER(I64)]
        L.lead_server_poll.argtypes = [P, I64, C.POINTER(I32)]
        L.lead_server_wait.argtypes = [P, I64]
        L.lead_server_result.argtypes = [P, I64, P, P, P, C.POINTER(I64), C.POINTER(I64)]
        L.lead_server_get_stats.argtypes = [P, C.POINTER(lead_server_stats)]
        L.lead_server_close.argtypes = [P]
        L.lead_server_clock_ns.argtypes = []
        L.lead_server_destroy.argtypes = [P]
        L.lead_server_destroy.restype = None
        for name in SYMBOLS:
            fn = getattr(L, name)
            if name == "lead_server_clock_ns":
                fn.restype = C.c_int64
            elif name not in ("lead_code_destroy", "lead_decoder_destroy", "lead_last_error",
                              "lead_batch_graph_destroy", "lead_batch_fused_destroy", "lead_server_destroy"):
                fn.restype = C.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != LEAD_OK:
        raise LeadError(status, lib().lead_last_error().decode())


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------------------
# C-named wrappers (argument marshalling only)
# ---------------------------------------------------------------------------

def lead_code_create(mul, delta, A, B, GA, GB):
    mul = np.ascontiguousarray(mul, dtype=np.uint16)
    A = np.ascontiguousarray(A, dtype=np.int32)
    B = np.ascontiguousarray(B, dtype=np.int32)
    GA = np.ascontiguousarray([int(x) for x in GA], dtype=np.uint64)
    GB = np.ascontiguousarray([int(x) for x in GB], dtype=np.uint64)
    desc = lead_code_desc(mul.shape[0], _np_ptr(mul), delta, _np_ptr(A), _np_ptr(B), len(GA), len(GB),
                          _np_ptr(GA), _np_ptr(GB))
    h = C.c_void_p()
    _check(lib().lead_code_create(C.byref(desc), C.byref(h)))
    return h


def lead_code_query(code) -> lead_code_info:
    info = lead_code_info()
    _check(lib().lead_code_query(code, C.byref(info)))
    return info


def lead_code_get_H(code, t, m):
    indptr = np.zeros(m + 1, dtype=np.int32)
    _check(lib().lead_code_get_H(code, t, _np_ptr(indptr), None))
    indices = np.zeros(int(indptr[-1]), dtype=np.int32)
    _check(lib().lead_code_get_H(code, t, _np_ptr(indptr), _np_ptr(indices)))
    return indptr, indices


def lead_code_get_views(code, t, order, d2):
    view = np.zeros((order, d2), dtype=np.int32)
    _check(lib().lead_code_get_views(code, t, _np_ptr(view)))
    return view


def lead_code_specialize(code, t):
    _check(lib().lead_code_specialize(code, t))


def lead_code_destroy(code):
    lib().lead_code_destroy(code)


def lead_params_make(alpha=1.0, ms_scale=0.75, max_iter_local=32, max_iter_global=32, llr_clamp=30.0,
                     early_exit=1, stage=LEAD_STAGE_FULL, boost=1, fixed_point_stop=1, local_post=0,
                     bp=LEAD_BP_MINSUM, global_post=0, osd_order=0) -> lead_params:
    return lead_params(alpha, ms_scale, max_iter_local, max_iter_global, llr_clamp, early_exit, stage, boost,
                       fixed_point_stop, local_post, bp, global_post, osd_order)


def lead_decoder_create(code, t, params: lead_params, max_shots: int):
    h = C.c_void_p()
    _check(lib().lead_decoder_create(code, t, C.byref(params), max_shots, C.byref(h)))
    return h


def lead_decoder_set_params(dec, params: lead_params):
    _check(lib().lead_decoder_set_params(dec, C.byref(params)))


def lead_decoder_set_schedule(dec, schedule: lead_schedule):
    _check(lib().lead_decoder_set_schedule(dec, C.byref(schedule)))


def lead_decoder_get_schedule(dec) -> lead_schedule:
    sc = lead_schedule()
    _check(lib().lead_decoder_get_schedule(dec, C.byref(sc)))
    return sc


def lead_decoder_destroy(dec):
    lib().lead_decoder_destroy(dec)


def lead_decode(dec, shots, synd, synd_words, prior, mode, ehat, ehat_words, post, lam, stats, stream):
    _check(lib().lead_decode(dec, shots, synd, synd_words, prior, mode, ehat, ehat_words, post, lam, stats,
                             stream))


def lead_decode_noalloc(dec, shots, synd, synd_words, prior, mode, ehat, ehat_words, post, lam, stats, stream):
    _check(lib().lead_decode_noalloc(dec, shots, synd, synd_words, prior, mode, ehat, ehat_words, post, lam,
                                     stats, stream))


def lead_decode_plain(dec, shots, synd, synd_words, prior, mode, ehat, ehat_words, post, lam, stats, stream):
    _check(lib().lead_decode_plain(dec, shots, synd, synd_words, prior, mode, ehat, ehat_words, post, lam,
                                   stats, stream))


def lead_syndrome(dec, shots, err, err_words, synd, synd_words, stream):
    _check(lib().lead_syndrome(dec, shots, err, err_words, synd, synd_words, stream))


def lead_decoder_autotune(dec, shots, synd, synd_words, prior, mode, stream) -> lead_schedule:
    best = lead_schedule()
    _check(lib().lead_decoder_autotune(dec, shots, synd, synd_words, prior, mode, stream, C.byref(best)))
    return best


def lead_batch_decode(items, stream):
    arr = (lead_batch_item * len(items))(*items)
    _check(lib().lead_batch_decode(arr, len(items), stream))


def lead_batch_graph_create(items, stream):
    arr = (lead_batch_item * len(items))(*items)
    g = C.c_void_p()
    _check(lib().lead_batch_graph_create(arr, len(items), stream, C.byref(g)))
    return g


def lead_batch_graph_launch(graph, stream):
    _check(lib().lead_batch_graph_launch(graph, stream))


def lead_batch_graph_destroy(graph):
    lib().lead_batch_graph_destroy(graph)


# ---------------------------------------------------------------------------
# torch-facing wrappers
# ---------------------------------------------------------------------------

def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, name, shape, dtype, optional=False):
    """Check a device tensor before its pointer crosses the C ABI (the
    library cannot see buffer sizes)."""
    if t is None:
        if optional:
            return
        raise ValueError(f"{name} is required")
    if str(t.dtype) != "torch." + dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous GPU tensor")
    if len(t.shape) != len(shape) or any(w is not None and w != g for w, g in zip(shape, t.shape)):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Code:
    """A quantum Tanner code built by the library from (G, A, B, C_A, C_B)."""

    def __init__(self, mul, delta, A, B, GA, GB):
        self._h = lead_code_create(mul, delta, A, B, GA, GB)
        self.info = lead_code_query(self._h)

    @classmethod
    def from_spec(cls, spec):
        return cls(spec.mul, spec.delta, spec.A, spec.B, spec.GA, spec.GB)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.lead_code_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def n(self):
        return self.info.n

    def m(self, t=LEAD_CHECK_Z):
        return self.info.m[t]

    def H(self, t=LEAD_CHECK_Z) -> np.ndarray:
        indptr, indices = lead_code_get_H(self._h, t, self.info.m[t])
        H = np.zeros((self.info.m[t], self.info.n), dtype=np.uint8)
        rows = np.repeat(np.arange(self.info.m[t]), np.diff(indptr))
        H[rows, indices] = 1
        return H

    def views(self, t=LEAD_CHECK_Z) -> np.ndarray:
        return lead_code_get_views(self._h, t, self.info.order, self.info.delta ** 2)

    def specialize(self, t=LEAD_CHECK_Z):
        """Compile (no GPU needed) the kernels specialised to check type t."""
        lead_code_specialize(self._h, t)


class Decoder:
    """LEAD decoder for one check type of a code, on the current device."""

    def __init__(self, code: Code, t=LEAD_CHECK_Z, max_shots=1 << 20, **params):
        self.code = code
        self.t = t
        self.params = lead_params_make(**params)
        self.max_shots = max_shots
        self._h = lead_decoder_create(code._h, t, self.params, max_shots)
        self.n = code.info.n
        self.m = code.info.m[t]
        self.synd_words = (self.m + 63) // 64
        self.ehat_words = (self.n + 63) // 64

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.lead_decoder_destroy(h)
            except Exception:
                pass
            self._h = None

    def set_params(self, **params):
        self.params = lead_params_make(**params)
        lead_decoder_set_params(self._h, self.params)

    def set_schedule(self, shots_per_workgroup=0, fused=0, local_chunk=0, local_waves=0, specialized=2,
                     chunk_shots=0, global_osd_form=0, global_tiles=0):
        lead_decoder_set_schedule(self._h, lead_schedule(shots_per_workgroup, fused, local_chunk, local_waves,
                                                         specialized, chunk_shots, global_osd_form, global_tiles))

    def get_schedule(self) -> dict:
        sc = lead_decoder_get_schedule(self._h)
        return {f: getattr(sc, f) for f, _ in lead_schedule._fields_}

    def time_phases(self, enable=True):
        """Switch per-phase device timing of the work-queue form on (clearing
        the sums) or off."""
        _check(lib().lead_decoder_time_phases(self._h, 1 if enable else 0))

    def phase_times(self) -> dict:
        """Summed device milliseconds and launch counts of Phase 1 and of
        Phases 2-3 since timing was switched on."""
        t = lead_phase_times()
        _check(lib().lead_decoder_phase_times(self._h, C.byref(t)))
        return {f: getattr(t, f) for f, _ in lead_phase_times._fields_}

    def alloc_outputs(self, shots, device="cuda", post=True, lam=False, stats=True):
        import torch
        out = dict(ehat=torch.empty((shots, self.ehat_words), dtype=torch.int64, device=device))
        out["post"] = torch.empty((shots, self.n), dtype=torch.float32, device=device) if post else None
        out["lam"] = torch.empty((shots, self.n), dtype=torch.float32, device=device) if lam else None
        out["stats"] = torch.empty((shots, 8), dtype=torch.int32, device=device) if stats else None
        return out

    def decode(self, synd, prior, mode=LEAD_PRIOR_PER_SHOT, out=None, post=True, lam=False, stream=None,
               plain=False, noalloc=False):
        """synd: int64 tensor [S, W] of packed syndromes on the GPU; prior:
        float32 LLRs ([S] PER_SHOT, [n] SHARED, [S, n] FULL).  Returns the
        dict of output tensors (ehat packed int64, post, lam, stats [S, 8]).
        plain: lead_decode_plain; noalloc: lead_decode_noalloc (the library's
        static scratch; pass `out` to allocate nothing on this side either)."""
        shots = int(synd.shape[0])
        _need(synd, "synd", (shots, None), "int64")
        if synd.shape[1] < self.synd_words:
            raise ValueError(f"synd has {synd.shape[1]} words per shot, need {self.synd_words}")
        want = {LEAD_PRIOR_PER_SHOT: (shots,), LEAD_PRIOR_SHARED: (self.n,), LEAD_PRIOR_FULL: (shots, self.n)}
        if mode not in want:
            raise ValueError("bad prior mode")
        _need(prior, "prior", want[mode], "float32")
        if out is None:
            out = self.alloc_outputs(shots, synd.device, post=post, lam=lam)
        _need(out["ehat"], "ehat", (shots, self.ehat_words), "int64", optional=True)
        _need(out["post"], "post", (shots, self.n), "float32", optional=True)
        _need(out["lam"], "lam", (shots, self.n), "float32", optional=True)
        _need(out["stats"], "stats", (shots, 8), "int32", optional=True)
        fn = lead_decode_plain if plain else lead_decode_noalloc if noalloc else lead_decode
        fn(self._h, shots, _ptr(synd), int(synd.shape[1]), _ptr(prior), mode, _ptr(out["ehat"]),
           self.ehat_words if out["ehat"] is not None else 0, _ptr(out["post"]), _ptr(out["lam"]),
           _ptr(out["stats"]), _stream(stream))
        return out

    def autotune(self, synd, prior, mode=LEAD_PRIOR_PER_SHOT, stream=None) -> dict:
        """Time the candidate schedules on this batch and keep the fastest."""
        shots = int(synd.shape[0])
        _need(synd, "synd", (shots, None), "int64")
        best = lead_decoder_autotune(self._h, shots, _ptr(synd), int(synd.shape[1]), _ptr(prior), mode,
                                     _stream(stream))
        return {f: getattr(best, f) for f, _ in lead_schedule._fields_}

    def batch_item(self, synd, prior, out, mode=LEAD_PRIOR_PER_SHOT) -> lead_batch_item:
        shots = int(synd.shape[0])
        _need(synd, "synd", (shots, None), "int64")
        _need(out["ehat"], "ehat", (shots, self.ehat_words), "int64", optional=True)
        _need(out["post"], "post", (shots, self.n), "float32", optional=True)
        _need(out["lam"], "lam", (shots, self.n), "float32", optional=True)
        _need(out["stats"], "stats", (shots, 8), "int32", optional=True)
        return lead_batch_item(self._h.value, shots, synd.data_ptr(), int(synd.shape[1]), prior.data_ptr(), mode,
                               out["ehat"].data_ptr() if out["ehat"] is not None else None, self.ehat_words,
                               out["post"].data_ptr() if out["post"] is not None else None,
                               out["lam"].data_ptr() if out["lam"] is not None else None,
                               out["stats"].data_ptr() if out["stats"] is not None else None)

    def syndrome(self, err, stream=None):
        import torch
        shots = int(err.shape[0])
        _need(err, "err", (shots, None), "int64")
        if err.shape[1] < self.ehat_words:
            raise ValueError(f"err has {err.shape[1]} words per shot, need {self.ehat_words}")
        synd = torch.empty((shots, self.synd_words), dtype=torch.int64, device=err.device)
        lead_syndrome(self._h, shots, _ptr(err), int(err.shape[1]), _ptr(synd), self.synd_words, _stream(stream))
        return synd


class Batch:
    """Several decode requests (possibly of different codes) decoded by one
    call, or captured once into a graph and replayed.  Each entry is
    (decoder, synd, prior, out, mode); the tensors must stay alive."""

    def __init__(self, entries):
        self.entries = list(entries)
        self.items = [dec.batch_item(synd, prior, out, mode) for dec, synd, prior, out, mode in self.entries]
        self._graph = None

    def run(self, stream=None):
        lead_batch_decode(self.items, _stream(stream))

    def capture(self, stream=None):
        if self._graph is None:
            self._graph = lead_batch_graph_create(self.items, _stream(stream))
        return self

    def replay(self, stream=None):
        if self._graph is None:
            self.capture(stream)
        lead_batch_graph_launch(self._graph, _stream(stream))

    def __del__(self):
        g = getattr(self, "_graph", None)
        if g and _lib is not None:
            try:
                _lib.lead_batch_graph_destroy(g)
            except Exception:
                pass
            self._graph = None


class FusedBatch:
    """Several decode requests (codes, check types, shot counts, priors)
    fused into one persistent Phase 1 launch and one Phases 2-3 launch,
    captured as a graph (lead_batch_fused_*).  entries: (decoder, synd,
    prior, out[, mode]) as for Batch; the buffers are bound at creation."""

    def __init__(self, entries):
        self._keep = list(entries)
        items = (lead_batch_item * len(entries))(*[e[0].batch_item(e[1], e[2], e[3], *e[4:]) for e in entries])
        h = C.c_void_p()
        _check(lib().lead_batch_fused_create(items, len(entries), C.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(lib().lead_batch_fused_launch(self._h, _stream(stream)))

    @staticmethod
    def specialize(parts):
        """Compile ahead of time: parts = [(Code, check type, form, prior mode)]."""
        n = len(parts)
        codes = (C.c_void_p * n)(*[p[0]._h.value for p in parts])
        types = np.array([p[1] for p in parts], dtype=np.int32)
        forms = np.array([p[2] for p in parts], dtype=np.int32)
        modes = np.array([p[3] for p in parts], dtype=np.int32)
        _check(lib().lead_batch_fused_specialize(codes, _np_ptr(types), _np_ptr(forms), _np_ptr(modes), n))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.lead_batch_fused_destroy(h)
            except Exception:
                pass
            self._h = None


class Server:
    """Continuous-batching request loop over a set of decoders (host
    requests in, host results out)."""

    def __init__(self, decoders, mem_budget_bytes=1 << 30, max_batch_shots=4096, max_slots_per_decoder=4,
                 return_posteriors=False, max_pending_shots=0):
        self.decoders = list(decoders)
        arr = (C.c_void_p * len(self.decoders))(*[d._h.value for d in self.decoders])
        cfg = lead_server_config(mem_budget_bytes, max_batch_shots, max_slots_per_decoder, int(return_posteriors), 0,
                                 max_pending_shots)
        self.return_posteriors = return_posteriors
        h = C.c_void_p()
        _check(lib().lead_server_create(arr, len(self.decoders), C.byref(cfg), C.byref(h)))
        self._h = h

    def submit(self, index: int, synd: np.ndarray, prior: np.ndarray) -> int:
        synd = np.ascontiguousarray(synd, dtype=np.uint64)
        prior = np.ascontiguousarray(prior, dtype=np.float32)
        if synd.ndim != 2 or prior.shape != (synd.shape[0],):
            raise ValueError("synd must be [shots, words] and prior [shots]")
        t = C.c_int64()
        _check(lib().lead_server_submit(self._h, index, synd.shape[0], _np_ptr(synd), synd.shape[1],
                                        _np_ptr(prior), C.byref(t)))
        return t.value

    def poll(self, ticket: int) -> bool:
        d = C.c_int32()
        _check(lib().lead_server_poll(self._h, ticket, C.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int):
        _check(lib().lead_server_wait(self._h, ticket))

    def result(self, ticket: int, index: int, shots: int) -> dict:
        dec = self.decoders[index]
        ehat = np.zeros((shots, dec.ehat_words), dtype=np.uint64)
        stats = np.zeros((shots, 8), dtype=np.int32)
        post = np.zeros((shots, dec.n), dtype=np.float32) if self.return_posteriors else None
        t0, t1 = C.c_int64(), C.c_int64()
        _check(lib().lead_server_result(self._h, ticket, _np_ptr(ehat), None if post is None else _np_ptr(post),
                                        _np_ptr(stats), C.byref(t0), C.byref(t1)))
        return dict(ehat=ehat, post=post, stats=stats, submit_ns=t0.value, done_ns=t1.value)

    def stats(self) -> dict:
        st = lead_server_stats()
        _check(lib().lead_server_get_stats(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in lead_server_stats._fields_}

    @staticmethod
    def clock_ns() -> int:
        return lib().lead_server_clock_ns()

    def drain(self):
        """lead_server_close: refuse new requests, wait for the admitted ones
        (their results stay available)."""
        _check(lib().lead_server_close(self._h))

    def close(self):
        """Finish the device work and free the server (lead_server_destroy)."""
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.lead_server_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
