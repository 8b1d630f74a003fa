"""Python binding of libsagms (argument marshalling only).

Every computation runs in the HIP kernels of ``libsagms.so``; this module
checks tensor shapes / dtypes / devices and passes raw device pointers and
the current HIP stream through the C ABI declared in ``include/sagms.h``.
PyTorch supplies device memory and streams.  Packed bit vectors (uint64
words in the ABI) are stored in int64 tensors.

Importing works without a GPU (graph construction is host code); the device
entry points raise if no GPU is present.  If ``libsagms.so`` has not been
built, loading raises ``ImportError`` -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SAGMS_LIBRARY may name another build of the same library (a sanitizer
# build of the host code, for instance); there is no other fallback.
LIB_PATH = os.environ.get("SAGMS_LIBRARY") or os.path.join(_HERE, "libsagms.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "sagms.h")

OK, EINVAL, ENOMEM, EUNSUPPORTED, EHIP = 0, -1, -2, -3, -4
KINDS = {"ms": 0, "sms": 1, "sagms": 2, "bp": 3}
PRECISIONS = {"fp32": 0, "fp16": 1, "int6": 2}
SCHEDULES = {"flooding": 0, "layered": 1}

_lib = None


class SagmsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libsagms error %d: %s" % (code, msg))
        self.code = code


class DecoderConfig(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("schedule", ctypes.c_int32), ("lmax", ctypes.c_int32),
                ("msg_precision", ctypes.c_int32), ("alpha", ctypes.c_double), ("alpha_min", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("eta", ctypes.c_double), ("frames_per_wave", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Segment(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_void_p), ("synd", ctypes.c_void_p), ("llr0", ctypes.c_void_p),
                ("nframes", ctypes.c_int64), ("ehat", ctypes.c_void_p), ("iters", ctypes.c_void_p),
                ("converged", ctypes.c_void_p), ("posterior", ctypes.c_void_p)]


PLAN_KINDS = {"single": 0, "tiered": 1, "per_code": 2}


class Plan(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("tile_frames", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("reg_budget", ctypes.c_int32), ("unroll", ctypes.c_int32)]

    def as_dict(self):
        kind = {v: k for k, v in PLAN_KINDS.items()}.get(self.kind, self.kind)
        return dict(kind=kind, tile_frames=self.tile_frames, waves_per_block=self.waves_per_block,
                    blocks_per_cu=self.blocks_per_cu, reg_budget=self.reg_budget, unroll=self.unroll)


class TuneResult(ctypes.Structure):
    _fields_ = [("plan", Plan), ("ms", ctypes.c_float)]


def plan(kind="single", tile_frames=8, waves_per_block=4, blocks_per_cu=0, reg_budget=0, unroll=1) -> Plan:
    if kind not in PLAN_KINDS:
        raise ValueError("unknown plan kind %r" % kind)
    return Plan(PLAN_KINDS[kind], int(tile_frames), int(waves_per_block), int(blocks_per_cu), int(reg_budget),
                int(unroll))


class GraphInfo(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in
                ("m", "n", "n_edges", "k", "dc_max", "dv_max", "words_n", "words_m", "joint", "words_e",
                 "layered_group", "layered_passes")]


def lib():
    """The loaded libsagms (raises ImportError when it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsagms.so is not built (python -m paper_2605_10433_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u32, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                       ctypes.c_uint64, ctypes.c_double)
        sigs = {
            "sagms_build_graph": [i32, i32, vp, vp, i32, vp, vp, vp],
            "sagms_build_gb": [i32, vp, i32, vp, i32, vp],
            "sagms_build_gb_joint": [i32, vp, i32, vp, i32, vp],
            "sagms_graph_info": [vp, vp],
            "sagms_graph_rows": [vp, vp],
            "sagms_graph_logicals": [vp, vp],
            "sagms_destroy_graph": [vp],
            "sagms_graph_upload": [vp],
            "sagms_gen_errors": [vp, u64, u32, u64, i64, dbl, vp, vp, vp, vp],
            "sagms_decode": [vp, vp, vp, vp, i64, vp, vp, vp, vp],
            "sagms_decode_soft": [vp, vp, vp, vp, i64, vp, vp, vp, vp, vp],
            "sagms_judge": [vp, vp, vp, vp, vp, i64, vp, vp, vp],
            "sagms_judge_joint": [vp, vp, vp, vp, vp, vp, i64, vp, vp, vp],
            "sagms_batch_create": [vp, i32, vp, vp],
            "sagms_batch_set_plan": [vp, vp],
            "sagms_batch_get_plan": [vp, vp],
            "sagms_batch_run": [vp, vp],
            "sagms_batch_instantiate": [vp],
            "sagms_batch_tune": [vp, vp, i32, vp, i32, vp, vp],
            "sagms_batch_destroy": [vp],
            "sagms_decode_segments": [vp, i32, vp, vp, vp],
            "sagms_server_create": [vp, vp, i32, vp, vp, vp],
            "sagms_server_submit": [vp, vp, vp],
            "sagms_server_progress": [vp, vp, i32, vp],
            "sagms_server_pending": [vp, vp, vp, vp],
            "sagms_server_replay": [vp, vp, vp, i64, dbl, vp],
            "sagms_server_destroy": [vp],
        }
        for name, args in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.sagms_last_error.argtypes = []
        L.sagms_last_error.restype = ctypes.c_char_p
        L.sagms_prior_llr.argtypes = [dbl]
        L.sagms_prior_llr.restype = ctypes.c_float
        L.sagms_depolarizing_llr.argtypes = [dbl]
        L.sagms_depolarizing_llr.restype = ctypes.c_float
        L.sagms_alpha_star.argtypes = [dbl, i32]
        L.sagms_alpha_star.restype = ctypes.c_double
        L.sagms_derive_gains.argtypes = [dbl, i32, dbl, dbl, vp]
        L.sagms_derive_gains.restype = ctypes.c_int
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared in include/sagms.h."""
    text = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"^\s*(?:int|float|const char\*)\s+(sagms_\w+)\s*\(", text, flags=re.M)))


def _check(rc):
    if rc != OK:
        raise SagmsError(rc, lib().sagms_last_error().decode())


def depolarizing_llr(p: float) -> float:
    """Prior log-ratio of a joint graph's variables, ln((1 - p) / (p / 3)), as float."""
    return float(lib().sagms_depolarizing_llr(float(p)))


def prior_llr(p: float) -> float:
    return float(lib().sagms_prior_llr(float(p)))


def alpha_star(l0: float, dc: int) -> float:
    return float(lib().sagms_alpha_star(float(l0), int(dc)))


def derived_config(l0, dc, ratio=0.6, eta=0.0, lmax=100, frames_per_wave=0, precision="fp32") -> "DecoderConfig":
    """SAGMS with the derived gains of sagms_derive_gains (eta <= 0: 1 / alpha_max)."""
    cfg = decoder_config("sagms", lmax=lmax, frames_per_wave=frames_per_wave, precision=precision)
    _check(lib().sagms_derive_gains(float(l0), int(dc), float(ratio), float(eta), ctypes.byref(cfg)))
    return cfg


def decoder_config(kind="sagms", lmax=100, alpha=0.75, alpha_min=0.30, alpha_max=0.50, eta=1.10,
                   frames_per_wave=0, precision="fp32", schedule="flooding") -> DecoderConfig:
    if kind not in KINDS:
        raise ValueError("unknown decoder kind %r" % kind)
    if precision not in PRECISIONS:
        raise ValueError("unknown message precision %r" % precision)
    if schedule not in SCHEDULES:
        raise ValueError("unknown schedule %r" % schedule)
    return DecoderConfig(KINDS[kind], SCHEDULES[schedule], int(lmax), PRECISIONS[precision], float(alpha),
                         float(alpha_min), float(alpha_max), float(eta), int(frames_per_wave), 0)


class Graph:
    """An immutable Tanner graph handle owned by libsagms."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)
        info = GraphInfo()
        _check(lib().sagms_graph_info(self._h, ctypes.byref(info)))
        for name, _ in GraphInfo._fields_:
            setattr(self, name, int(getattr(info, name)))

    @classmethod
    def gb(cls, l, a, b):
        a = np.ascontiguousarray(a, dtype=np.int32)
        b = np.ascontiguousarray(b, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(lib().sagms_build_gb(int(l), a.ctypes.data, len(a), b.ctypes.data, len(b), ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def gb_joint(cls, l, a, b):
        """The joint (quaternary) graph of a GB code: X-type rows of H_X, then
        Z-type rows of H_Z (sagms_build_gb_joint)."""
        a = np.ascontiguousarray(a, dtype=np.int32)
        b = np.ascontiguousarray(b, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(lib().sagms_build_gb_joint(int(l), a.ctypes.data, len(a), b.ctypes.data, len(b), ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def from_dense(cls, h, h_other=None):
        def csr(mat):
            mat = np.asarray(mat, dtype=np.uint8)
            rp = np.zeros(mat.shape[0] + 1, dtype=np.int32)
            cols = []
            for i, row in enumerate(mat):
                nz = np.nonzero(row & 1)[0]
                cols.extend(nz.tolist())
                rp[i + 1] = len(cols)
            return rp, np.asarray(cols, dtype=np.int32)
        h = np.asarray(h)
        rp, ci = csr(h)
        hdl = ctypes.c_void_p()
        if h_other is None:
            _check(lib().sagms_build_graph(h.shape[0], h.shape[1], rp.ctypes.data, ci.ctypes.data, 0, None, None,
                                           ctypes.byref(hdl)))
        else:
            rpo, cio = csr(h_other)
            _check(lib().sagms_build_graph(h.shape[0], h.shape[1], rp.ctypes.data, ci.ctypes.data,
                                           np.asarray(h_other).shape[0], rpo.ctypes.data, cio.ctypes.data,
                                           ctypes.byref(hdl)))
        return cls(hdl.value)

    def rows(self) -> np.ndarray:
        out = np.zeros((self.m, self.words_e), dtype=np.uint64)
        _check(lib().sagms_graph_rows(self._h, out.ctypes.data))
        return out

    def logicals(self) -> np.ndarray:
        rows = max(self.k, 0) * (2 if self.joint else 1)
        out = np.zeros((rows, self.words_e), dtype=np.uint64)
        _check(lib().sagms_graph_logicals(self._h, out.ctypes.data))
        return out

    def upload(self):
        """Copies the device tables to the current HIP device (the builders
        already do so for the device current when they run)."""
        _check(lib().sagms_graph_upload(self._h))

    def close(self):
        if self._h is not None and self._h.value:
            lib().sagms_destroy_graph(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- device entry points ------------------------------------------------
def _dev_ptr(t, dtype, shape, name):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must have dtype %s (got %s)" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s (got %s)" % (name, tuple(shape), tuple(t.shape)))
    return t.data_ptr()


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def gen_errors(g: Graph, seed, stream_id, frame0, nframes, p, ex, ez, synd, stream=None):
    import torch
    _check(lib().sagms_gen_errors(
        g._h, int(seed), int(stream_id), int(frame0), int(nframes), float(p),
        _dev_ptr(ex, torch.int64, (nframes, g.words_n), "ex"),
        _dev_ptr(ez, torch.int64, (nframes, g.words_n), "ez"),
        _dev_ptr(synd, torch.int64, (nframes, g.words_m), "synd"), _stream(stream)))


def decode(g: Graph, synd, llr0, cfg: DecoderConfig, ehat, iters, converged, stream=None):
    import torch
    nframes = synd.shape[0]
    _check(lib().sagms_decode(
        g._h, _dev_ptr(synd, torch.int64, (nframes, g.words_m), "synd"),
        _dev_ptr(llr0, torch.float32, (g.n,), "llr0"), ctypes.byref(cfg), int(nframes),
        _dev_ptr(ehat, torch.int64, (nframes, g.words_e), "ehat"),
        _dev_ptr(iters, torch.int32, (nframes,), "iters"),
        _dev_ptr(converged, torch.uint8, (nframes,), "converged"), _stream(stream)))


def decode_soft(g: Graph, synd, llr0, cfg: DecoderConfig, ehat, iters, converged, posterior, stream=None):
    import torch
    nframes = synd.shape[0]
    _check(lib().sagms_decode_soft(
        g._h, _dev_ptr(synd, torch.int64, (nframes, g.words_m), "synd"),
        _dev_ptr(llr0, torch.float32, (g.n,), "llr0"), ctypes.byref(cfg), int(nframes),
        _dev_ptr(ehat, torch.int64, (nframes, g.words_e), "ehat"),
        _dev_ptr(iters, torch.int32, (nframes,), "iters"),
        _dev_ptr(converged, torch.uint8, (nframes,), "converged"),
        _dev_ptr(posterior, torch.float32, (nframes, g.n, 3) if g.joint else (nframes, g.n), "posterior"),
        _stream(stream)))


def judge(g: Graph, ex, ehat, converged, iters, counters, fail=None, stream=None):
    import torch
    nframes = ex.shape[0]
    _check(lib().sagms_judge(
        g._h, _dev_ptr(ex, torch.int64, (nframes, g.words_n), "ex"),
        _dev_ptr(ehat, torch.int64, (nframes, g.words_n), "ehat"),
        _dev_ptr(converged, torch.uint8, (nframes,), "converged"),
        _dev_ptr(iters, torch.int32, (nframes,), "iters"), int(nframes),
        _dev_ptr(fail, torch.uint8, (nframes,), "fail"),
        _dev_ptr(counters, torch.int64, (2,), "counters"), _stream(stream)))


def judge_joint(g: Graph, ex, ez, ehat, converged, iters, counters, fail=None, stream=None):
    """The judge of a joint graph (sagms_judge_joint)."""
    import torch
    nframes = ex.shape[0]
    _check(lib().sagms_judge_joint(
        g._h, _dev_ptr(ex, torch.int64, (nframes, g.words_n), "ex"),
        _dev_ptr(ez, torch.int64, (nframes, g.words_n), "ez"),
        _dev_ptr(ehat, torch.int64, (nframes, g.words_e), "ehat"),
        _dev_ptr(converged, torch.uint8, (nframes,), "converged"),
        _dev_ptr(iters, torch.int32, (nframes,), "iters"), int(nframes),
        _dev_ptr(fail, torch.uint8, (nframes,), "fail"),
        _dev_ptr(counters, torch.int64, (2,), "counters"), _stream(stream)))


def frame_buffers(g: Graph, nframes: int, device="cuda", with_ez=True):
    """Device tensors for one batch: ex, ez, synd, ehat, iters, converged, fail."""
    import torch
    z = dict(device=device)
    return dict(
        ex=torch.empty((nframes, g.words_n), dtype=torch.int64, **z),
        ez=torch.empty((nframes, g.words_n), dtype=torch.int64, **z) if with_ez else None,
        synd=torch.empty((nframes, g.words_m), dtype=torch.int64, **z),
        ehat=torch.empty((nframes, g.words_e), dtype=torch.int64, **z),
        iters=torch.empty((nframes,), dtype=torch.int32, **z),
        converged=torch.empty((nframes,), dtype=torch.uint8, **z),
        fail=torch.empty((nframes,), dtype=torch.uint8, **z),
    )


def _segment_array(segments):
    """The sagms_segment array of a list of segment dicts (see Batch)."""
    import torch
    n = len(segments)
    arr = (Segment * max(n, 1))()
    for i, sg in enumerate(segments):
        g = sg["graph"]
        nf = int(sg["synd"].shape[0])
        arr[i].graph = g._h.value if g is not None else None
        arr[i].synd = _dev_ptr(sg["synd"], torch.int64, (nf, g.words_m), "synd")
        arr[i].llr0 = _dev_ptr(sg["llr0"], torch.float32, (g.n,), "llr0")
        arr[i].nframes = nf
        arr[i].ehat = _dev_ptr(sg["ehat"], torch.int64, (nf, g.words_n), "ehat")
        arr[i].iters = _dev_ptr(sg["iters"], torch.int32, (nf,), "iters")
        arr[i].converged = _dev_ptr(sg["converged"], torch.uint8, (nf,), "converged")
        arr[i].posterior = _dev_ptr(sg.get("posterior"), torch.float32, (nf, g.n), "posterior")
    return arr, n


def decode_segments(segments, cfg: DecoderConfig, plan_: Plan = None, stream=None):
    """One mixed-code decode without a batch object or any allocation
    (``sagms_decode_segments``); segments as for Batch."""
    arr, n = _segment_array(segments)
    _check(lib().sagms_decode_segments(ctypes.cast(arr, ctypes.c_void_p), n, ctypes.byref(cfg),
                                       ctypes.byref(plan_) if plan_ is not None else None, _stream(stream)))


class Batch:
    """A mixed-code batch (``sagms_batch_*``).

    ``segments`` is a list of dicts with keys graph, synd, llr0, ehat, iters,
    converged and optionally posterior (device tensors shaped as for
    ``decode``).  The tensors are referenced by the batch: they must stay
    alive, and in place, as long as it does.
    """

    def __init__(self, segments, cfg: DecoderConfig):
        arr, n = _segment_array(segments)
        self._keep = list(segments)
        self._cfg = cfg
        h = ctypes.c_void_p()
        _check(lib().sagms_batch_create(ctypes.cast(arr, ctypes.c_void_p), n, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    def set_plan(self, p: Plan):
        _check(lib().sagms_batch_set_plan(self._h, ctypes.byref(p)))

    def get_plan(self) -> Plan:
        p = Plan()
        _check(lib().sagms_batch_get_plan(self._h, ctypes.byref(p)))
        return p

    def run(self, stream=None):
        _check(lib().sagms_batch_run(self._h, _stream(stream)))

    def instantiate(self):
        _check(lib().sagms_batch_instantiate(self._h))

    def tune(self, reps=3, stream=None, cap=256):
        """Runs the autotuner; returns (best plan, [(plan dict, ms), ...])."""
        res = (TuneResult * cap)()
        cnt = ctypes.c_int32()
        best = Plan()
        _check(lib().sagms_batch_tune(self._h, _stream(stream), int(reps), ctypes.cast(res, ctypes.c_void_p), cap,
                                      ctypes.byref(cnt), ctypes.byref(best)))
        return best, [(res[i].plan.as_dict(), float(res[i].ms)) for i in range(cnt.value)]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sagms_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- serving ---------------------------------------------------------------
class ServerConfig(ctypes.Structure):
    _fields_ = [("max_frames_in_flight", ctypes.c_int64), ("max_frames_per_launch", ctypes.c_int32),
                ("min_launch_frames", ctypes.c_int32), ("max_wait_us", ctypes.c_double),
                ("streams", ctypes.c_int32), ("tile_frames", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("reg_budget", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("code", ctypes.c_int32), ("nframes", ctypes.c_int32), ("synd", ctypes.c_void_p),
                ("ehat", ctypes.c_void_p), ("iters", ctypes.c_void_p), ("converged", ctypes.c_void_p),
                ("deadline_us", ctypes.c_double)]


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("submit_us", ctypes.c_double), ("admit_us", ctypes.c_double), ("done_us", ctypes.c_double)]


REQ_DONE, REQ_CANCELLED = 0, 1
# NumPy views of the C structures, for traces of millions of requests
REQUEST_DTYPE = np.dtype({"names": ["code", "nframes", "synd", "ehat", "iters", "converged", "deadline_us"],
                          "formats": [np.int32, np.int32, np.uint64, np.uint64, np.uint64, np.uint64, np.float64],
                          "offsets": [0, 4, 8, 16, 24, 32, 40], "itemsize": 48})
COMPLETION_DTYPE = np.dtype({"names": ["id", "status", "reserved", "submit_us", "admit_us", "done_us"],
                             "formats": [np.int64, np.int32, np.int32, np.float64, np.float64, np.float64],
                             "offsets": [0, 8, 12, 16, 24, 32], "itemsize": 40})


def server_config(max_frames_in_flight=1 << 20, max_frames_per_launch=1 << 16, min_launch_frames=0, max_wait_us=0.0,
                  streams=4, tile_frames=8, waves_per_block=4, reg_budget=1) -> ServerConfig:
    return ServerConfig(int(max_frames_in_flight), int(max_frames_per_launch), int(min_launch_frames),
                        float(max_wait_us), int(streams), int(tile_frames), int(waves_per_block), int(reg_budget))


class Server:
    """A serving runtime over several codes (``sagms_server_*``).

    Requests carry host NumPy buffers: syndromes uint64 [nframes, words_m],
    outputs ehat uint64 [nframes, words_n], iters int32 [nframes], converged
    uint8 [nframes].  The caller keeps them alive until completion.
    """

    def __init__(self, graphs, priors, cfg: DecoderConfig, scfg: ServerConfig = None):
        self.graphs = list(graphs)
        self._priors = [np.ascontiguousarray(p, dtype=np.float32) for p in priors]
        for g, p in zip(self.graphs, self._priors):
            if p.shape != (g.n,):
                raise ValueError("prior of shape %s for a code with n = %d" % (p.shape, g.n))
        n = len(self.graphs)
        gh = (ctypes.c_void_p * max(n, 1))(*[g._h.value for g in self.graphs])
        ph = (ctypes.c_void_p * max(n, 1))(*[p.ctypes.data for p in self._priors])
        self._cfg = cfg
        self._scfg = scfg if scfg is not None else server_config()
        h = ctypes.c_void_p()
        _check(lib().sagms_server_create(ctypes.cast(gh, ctypes.c_void_p), ctypes.cast(ph, ctypes.c_void_p), n,
                                         ctypes.byref(cfg), ctypes.byref(self._scfg), ctypes.byref(h)))
        self._h = h

    @staticmethod
    def _check_buffers(g, synd, ehat, iters, converged):
        nf = synd.shape[0]
        for arr, dt, shape, name in ((synd, np.uint64, (nf, g.words_m), "synd"), (ehat, np.uint64, (nf, g.words_n), "ehat"),
                                     (iters, np.int32, (nf,), "iters"), (converged, np.uint8, (nf,), "converged")):
            if arr.dtype != dt or arr.shape != shape or not arr.flags["C_CONTIGUOUS"]:
                raise ValueError("%s must be a C-contiguous %s array of shape %s" % (name, np.dtype(dt), shape))
        return nf

    def submit(self, code, synd, ehat, iters, converged, deadline_us=0.0):
        nf = self._check_buffers(self.graphs[code], synd, ehat, iters, converged)
        r = Request(int(code), int(nf), synd.ctypes.data, ehat.ctypes.data, iters.ctypes.data, converged.ctypes.data,
                    float(deadline_us))
        rid = ctypes.c_int64()
        _check(lib().sagms_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)))
        return rid.value

    def progress(self, cap=1024):
        out = np.zeros(cap, dtype=COMPLETION_DTYPE)
        n = ctypes.c_int32()
        _check(lib().sagms_server_progress(self._h, out.ctypes.data, cap, ctypes.byref(n)))
        return out[:n.value]

    def pending(self):
        q, f, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().sagms_server_pending(self._h, ctypes.byref(q), ctypes.byref(f), ctypes.byref(c)))
        return q.value, f.value, c.value

    def replay(self, requests, arrival_us, timeout_s=30.0):
        """requests: REQUEST_DTYPE array (pointers to live host buffers);
        arrival_us: float64 [n], non-decreasing.  Returns COMPLETION_DTYPE [n]."""
        requests = np.ascontiguousarray(requests, dtype=REQUEST_DTYPE)
        arrival_us = np.ascontiguousarray(arrival_us, dtype=np.float64)
        if arrival_us.shape != (len(requests),):
            raise ValueError("one arrival time per request")
        out = np.zeros(len(requests), dtype=COMPLETION_DTYPE)
        _check(lib().sagms_server_replay(self._h, requests.ctypes.data, arrival_us.ctypes.data, len(requests),
                                         float(timeout_s), out.ctypes.data))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sagms_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
