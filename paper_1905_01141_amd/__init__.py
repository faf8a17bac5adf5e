"""Python binding of libtdec, the MI355X (gfx950) LTE turbo decoder.

Argument marshalling only: every step of the decoding path runs in the HIP
kernels of libtdec.so (see include/tdec.h for the C ABI and its contract).
PyTorch supplies device memory and the stream.  Importing works without a
GPU; any call that needs the library raises if libtdec.so is missing or no
GPU is present -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import functools
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdec.so")

CRC_NONE, CRC24A, CRC24B = 0, 1, 2
STATUS = {0: "OK", -1: "EINVAL", -2: "ERANGE", -3: "ENOMEM", -4: "EDEVICE", -5: "EBUSY"}
EXPORTS = ("tdec_segment", "tdec_tb_llr_count", "tdec_k_table", "tdec_qpp", "tdec_create",
           "tdec_destroy", "tdec_pick_windows", "tdec_set_max_windows", "cb_decode_batch", "cb_decode_batch_fixed",
           "tb_decode", "tb_decode_batch",
           "cb_encode_batch", "tb_encode", "tdec_now_ns", "tdec_server_create",
           "tdec_server_create_model", "tdec_server_submit", "tdec_server_poll",
           "tdec_server_drain", "tdec_server_stats", "tdec_server_reset_stats",
           "tdec_server_destroy", "tdec_graph_cb_decode", "tdec_graph_tb_decode",
           "tdec_graph_launch", "tdec_graph_destroy", "tdec_autotune", "tdec_autotune_reset",
           "tdec_server_submit_dev", "tdec_derate_batch", "tdec_rate_match_batch",
           "tdec_server_launches", "tdec_probe_valu_int16", "tdec_probe_hbm",
           "tdec_probe_launch", "tdec_server_replay", "tdec_default_knobs", "tdec_set_knobs",
           "tdec_get_knobs", "tdec_autotune_batch")
ORDER_K_DESC, ORDER_K_ASC, ORDER_REQUEST = 0, 1, 2
SERVE_CONTINUOUS, SERVE_PER_TB, SERVE_RING = 0, 1, 2
ADMIT_BUDGET, ADMIT_DEADLINE = 1, 2
SERVE_DONE, SERVE_REJ_BUDGET, SERVE_REJ_DEADLINE, SERVE_REJ_INVALID, SERVE_ERROR = 0, 1, 2, 3, 4


class TdecError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {STATUS.get(code, code)}")
        self.code = code


class Params(ct.Structure):
    _fields_ = [("max_iters", ct.c_int32), ("early_stop", ct.c_int32),
                ("n_windows", ct.c_int32), ("win_init", ct.c_int32),
                ("mi_eps", ct.c_int32)]


class Knobs(ct.Structure):
    _fields_ = [("lds_budget", ct.c_int32), ("order", ct.c_int32), ("win_target", ct.c_int32),
                ("grid_cap", ct.c_int32), ("us", ct.c_float)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Seg(ct.Structure):
    _fields_ = [(n, ct.c_int32) for n in
                ("B", "C", "L", "Kplus", "Kminus", "Cplus", "Cminus", "F")]


class CbDesc(ct.Structure):
    _fields_ = [("llr_off", ct.c_int64), ("bits_off", ct.c_int64), ("K", ct.c_int32),
                ("F", ct.c_int16), ("crc", ct.c_int8), ("rsv", ct.c_int8)]


class ServerCfg(ct.Structure):
    _fields_ = [("slot_budget_bytes", ct.c_size_t), ("deadline_us", ct.c_int32),
                ("max_batch_cb", ct.c_int32), ("mode", ct.c_int32), ("admission", ct.c_int32),
                ("model_lat_ns", ct.c_int64), ("model_ns_per_kbit", ct.c_int64),
                ("params", Params), ("max_inflight", ct.c_int32), ("ring_idle_us", ct.c_int32)]


class ServeResult(ct.Structure):
    _fields_ = [("tag", ct.c_uint64), ("tbs", ct.c_int32), ("status", ct.c_int32),
                ("tb_ok", ct.c_int32), ("max_iters_used", ct.c_int32), ("C", ct.c_int32),
                ("batch_tbs", ct.c_int32), ("t_arrive_ns", ct.c_int64), ("t_done_ns", ct.c_int64)]


class ServeStats(ct.Structure):
    _fields_ = [(n, ct.c_int64) for n in (
        "submitted", "admitted", "rej_budget", "rej_deadline", "rej_invalid", "completed",
        "tb_fail", "deadline_miss", "batches", "payload_bits", "busy_ns", "lat_p50_ns",
        "lat_p99_ns", "lat_p999_ns", "lat_max_ns", "lat_mean_ns", "model_lat_ns",
        "model_ns_per_kbit", "slots_in_use_bytes", "slots_peak_bytes", "mean_pre_ns",
        "mean_coding_ns", "mean_post_ns")] + [
        ("mean_batch_tbs", ct.c_double), ("mean_batch_cbs", ct.c_double),
        ("ring_launches", ct.c_int64), ("ring_grid", ct.c_int64)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


class LaunchRec(ct.Structure):
    _fields_ = [(n, ct.c_int64) for n in (
        "t_start_ns", "t_end_ns", "pre_ns", "coding_ns", "post_ns", "copy_ns",
        "oldest_wait_ns")] + [
        ("n_tb", ct.c_int32), ("n_cb", ct.c_int32), ("cb_bits", ct.c_int64),
        ("copyout_ns", ct.c_int64)]


class RmDesc(ct.Structure):
    _fields_ = [("e_off", ct.c_int64), ("soft_off", ct.c_int64), ("K", ct.c_int32),
                ("F", ct.c_int16), ("rv", ct.c_int8), ("rsv", ct.c_int8), ("E", ct.c_int32),
                ("Ncb", ct.c_int32)]


def rm_kw(K: int) -> int:
    """Circular buffer length of rate matching: 3 * 32 * ceil((K+4)/32)."""
    return 3 * 32 * ((int(K) + 4 + 31) // 32)


def make_rm_descs(blocks):
    """blocks: [(K, F, rv, E)] -> (descs, total E, soft elements), laid out
    back to back."""
    d = (RmDesc * len(blocks))()
    eo = so = 0
    for i, (K, F, rv, E) in enumerate(blocks):
        d[i].e_off, d[i].soft_off, d[i].K, d[i].F, d[i].rv, d[i].E, d[i].Ncb = eo, so, K, F, rv, E, 0
        eo += E
        so += 3 * (K + 4)
    return d, eo, so


# tdec_cb_desc as a numpy record (same layout) for vectorised checks
DESC_DTYPE = np.dtype([("llr_off", "<i8"), ("bits_off", "<i8"), ("K", "<i4"), ("F", "<i2"),
                       ("crc", "i1"), ("rsv", "i1")])

# tdec_tb_result as stored in device memory
TB_RESULT_DTYPE = np.dtype([("tb_ok", "<i4"), ("max_iters_used", "<i4"), ("C", "<i4"),
                            ("rsv", "<i4"), ("cb_ok", "u1", (64,)), ("cb_iters", "u1", (64,))])
TB_RESULT_BYTES = TB_RESULT_DTYPE.itemsize

_lib = None


def lib():
    """Load libtdec.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1905_01141_amd.build`")
        L = ct.CDLL(LIB_PATH)
        P, vp, i32, i64 = ct.POINTER, ct.c_void_p, ct.c_int32, ct.c_int64
        L.tdec_segment.argtypes = [i32, P(Seg)]
        L.tdec_tb_llr_count.restype = i64
        L.tdec_tb_llr_count.argtypes = [i32]
        L.tdec_k_table.argtypes = [vp]
        L.tdec_qpp.argtypes = [i32, vp, vp, vp]
        L.tdec_create.argtypes = [ct.c_int, ct.c_size_t, P(vp)]
        L.tdec_destroy.argtypes = [vp]
        L.tdec_destroy.restype = None
        L.tdec_pick_windows.argtypes = [vp, i32]
        L.tdec_set_max_windows.argtypes = [vp, i32]
        L.cb_decode_batch.argtypes = [vp, i32, vp, vp, P(Params), vp, vp, vp, vp]
        L.cb_decode_batch_fixed.argtypes = [vp, i32, vp, vp, P(Params), vp, vp, vp, vp]
        L.tb_decode.argtypes = [vp, vp, i32, P(Params), vp, vp, vp]
        L.tb_decode_batch.argtypes = [vp, i32, vp, vp, vp, vp, P(Params), vp, vp, vp]
        L.cb_encode_batch.argtypes = [vp, i32, vp, vp, vp, vp]
        L.tb_encode.argtypes = [vp, vp, i32, vp, vp]
        L.tdec_graph_cb_decode.argtypes = [vp, i32, vp, vp, P(Params), vp, vp, vp, P(vp)]
        L.tdec_graph_tb_decode.argtypes = [vp, i32, vp, vp, vp, vp, P(Params), vp, vp, P(vp)]
        L.tdec_graph_launch.argtypes = [vp, vp]
        L.tdec_graph_destroy.argtypes = [vp]
        L.tdec_graph_destroy.restype = None
        L.tdec_autotune.argtypes = [vp, i32, vp, i32, i32, i64, vp, vp, vp]
        L.tdec_autotune_reset.argtypes = [vp]
        L.tdec_autotune_reset.restype = None
        L.tdec_default_knobs.argtypes = [P(Knobs)]
        L.tdec_default_knobs.restype = None
        L.tdec_set_knobs.argtypes = [vp, P(Knobs)]
        L.tdec_get_knobs.argtypes = [vp, P(Knobs)]
        L.tdec_autotune_batch.argtypes = [vp, i32, vp, vp, vp, P(Params), i32, vp, i32, vp,
                                          P(Knobs), P(Knobs), vp]
        L.tdec_derate_batch.argtypes = [vp, i32, vp, vp, i32, vp, i32, vp]
        L.tdec_rate_match_batch.argtypes = [vp, i32, vp, vp, vp, vp]
        L.tdec_now_ns.restype = i64
        L.tdec_now_ns.argtypes = []
        L.tdec_server_create.argtypes = [vp, P(ServerCfg), P(vp)]
        L.tdec_server_create_model.argtypes = [P(ServerCfg), i64, i64, P(vp)]
        L.tdec_server_submit.argtypes = [vp, i32, vp, vp, vp, vp, i64, vp]
        L.tdec_server_submit_dev.argtypes = [vp, i32, vp, vp, vp, vp, i64, vp]
        L.tdec_server_poll.argtypes = [vp, vp, i32, i32]
        L.tdec_server_replay.argtypes = [vp, i32, i64, i64, vp, vp, vp, vp, ct.c_uint64, vp, vp]
        L.tdec_server_drain.argtypes = [vp, i32]
        L.tdec_server_stats.argtypes = [vp, P(ServeStats)]
        L.tdec_server_reset_stats.argtypes = [vp]
        L.tdec_server_reset_stats.restype = None
        L.tdec_server_destroy.argtypes = [vp]
        L.tdec_server_destroy.restype = None
        L.tdec_server_launches.argtypes = [vp, vp, i32]
        dp = P(ct.c_double)
        L.tdec_probe_valu_int16.argtypes = [ct.c_int, i32, dp]
        L.tdec_probe_hbm.argtypes = [ct.c_int, ct.c_size_t, dp, dp]
        L.tdec_probe_launch.argtypes = [ct.c_int, i32, dp, dp]
        _lib = L
    return _lib


def _check(fn, code):
    if code != 0:
        raise TdecError(fn, code)


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _dptr(t):
    """Device pointer of a torch CUDA tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ct.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


# ----------------------------------------------------------------------------- helpers
STOP_CRC, STOP_MI, STOP_PURGE = 1, 2, 4  # bits of Params.early_stop
MI_EPS_DEFAULT = 1         # 2^-15 bit per bit: looser thresholds stop max-log-MAP blocks
                           # whose a-posteriori values are large but still wrong


def params(max_iters=6, early_stop=0, n_windows=1, win_init=0, mi_eps=MI_EPS_DEFAULT) -> Params:
    """Decoder parameters (tdec_params).  early_stop: 0, or an OR of STOP_CRC,
    STOP_MI and STOP_PURGE (transport block calls); mi_eps: the STOP_MI
    threshold."""
    return Params(max_iters, early_stop, n_windows, win_init, mi_eps)


def probe_valu_int16(device: int = 0, iters: int = 20000) -> float:
    """Measured packed int16 VALU rate, TOP/s (include/tdec_probe.h)."""
    v = ct.c_double()
    _check("tdec_probe_valu_int16", lib().tdec_probe_valu_int16(device, iters, ct.byref(v)))
    return v.value


def probe_hbm(device: int = 0, nbytes: int = 1 << 30) -> tuple[float, float]:
    """Measured HBM (read GB/s, copy GB/s counting read + write)."""
    r, c = ct.c_double(), ct.c_double()
    _check("tdec_probe_hbm", lib().tdec_probe_hbm(device, nbytes, ct.byref(r), ct.byref(c)))
    return r.value, c.value


def probe_launch(device: int = 0, n: int = 2000) -> tuple[float, float]:
    """Device microseconds per back-to-back empty launch and per graph node."""
    a, b = ct.c_double(), ct.c_double()
    _check("tdec_probe_launch", lib().tdec_probe_launch(device, n, ct.byref(a), ct.byref(b)))
    return a.value, b.value


def segment(tbs: int) -> dict:
    s = Seg()
    _check("tdec_segment", lib().tdec_segment(int(tbs), ct.byref(s)))
    return {n: getattr(s, n) for n, _ in Seg._fields_}


def win_len(K: int, n_windows: int) -> int:
    """Trellis steps of every window but the last for a block of K bits in
    n_windows windows (include/tdec.h): K for one window, else
    8 * ceil(K / (8 * n_windows))."""
    K, n = int(K), int(n_windows)
    return K if n == 1 else 8 * (-(-K // (8 * n)))


def cb_sizes(tbs: int) -> list[tuple[int, int]]:
    s = segment(tbs)
    return [(s["Kminus"] if r < s["Cminus"] else s["Kplus"], s["F"] if r == 0 else 0)
            for r in range(s["C"])]


@functools.lru_cache(maxsize=4096)
def tb_llr_count(tbs: int) -> int:
    n = lib().tdec_tb_llr_count(int(tbs))
    if n < 0:
        raise TdecError("tdec_tb_llr_count", -2)
    return int(n)


def k_table() -> np.ndarray:
    out = np.zeros(188, np.int32)
    lib().tdec_k_table(_np_ptr(out))
    return out


def qpp(K: int) -> tuple[np.ndarray, int, int]:
    pi = np.zeros(K, np.int32)
    f1, f2 = ct.c_int32(), ct.c_int32()
    _check("tdec_qpp", lib().tdec_qpp(int(K), _np_ptr(pi), ct.byref(f1), ct.byref(f2)))
    return pi, f1.value, f2.value


def make_descs(cbs) -> tuple[ct.Array, int, int]:
    """Descriptor array for (K, F, crc) code blocks laid out back to back.
    Returns (descs, total LLR elements, total payload bytes)."""
    descs = (CbDesc * len(cbs))()
    llr_off = bits_off = 0
    for i, (K, F, crc) in enumerate(cbs):
        descs[i].llr_off, descs[i].bits_off = llr_off, bits_off
        descs[i].K, descs[i].F, descs[i].crc = int(K), int(F), int(crc)
        llr_off += 3 * (K + 4)
        L = 0 if crc == CRC_NONE else 24
        bits_off += (K - F - L + 7) // 8
    return descs, llr_off, bits_off


# tdec_rm_desc as a numpy record (same layout)
RM_DESC_DTYPE = np.dtype([("e_off", "<i8"), ("soft_off", "<i8"), ("K", "<i4"), ("F", "<i2"),
                          ("rv", "i1"), ("rsv", "i1"), ("E", "<i4"), ("Ncb", "<i4")])


def _rm_extent(descs):
    """(transmitted values, soft-buffer elements) a rate matching descriptor
    array reaches, vectorised."""
    v = np.frombuffer(descs, dtype=RM_DESC_DTYPE, count=len(descs))
    K = v["K"].astype(np.int64)
    return int((v["e_off"] + v["E"]).max()), int((v["soft_off"] + 3 * (K + 4)).max())


def _desc_extent(descs):
    """(LLR elements, payload bytes) a descriptor array reaches, vectorised."""
    if len(descs) == 0:
        return 0, 0
    v = np.frombuffer(descs, dtype=DESC_DTYPE, count=len(descs))
    K = v["K"].astype(np.int64)
    L = np.where(v["crc"] == CRC_NONE, 0, 24)
    nb = np.maximum(0, (K - v["F"] - L + 7) // 8)
    return int((v["llr_off"] + 3 * (K + 4)).max()), int((v["bits_off"] + nb).max())


def _need(t, dtype: str, n: int, name: str):
    """Check that device tensor t has the dtype and at least n elements, so
    that no descriptor can make a kernel reach past the buffer."""
    if t is None:
        raise ValueError(f"{name}: tensor required")
    if str(t.dtype) != "torch." + dtype:
        raise ValueError(f"{name}: {dtype} tensor expected, got {t.dtype}")
    if t.numel() < n:
        raise ValueError(f"{name}: {n} elements needed, tensor has {t.numel()}")


# ----------------------------------------------------------------------------- context
class Decoder:
    """A libtdec context on one GPU (owns the device workspace)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.device = device
        h = ct.c_void_p()
        _check("tdec_create", lib().tdec_create(device, hbm_budget_bytes, ct.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().tdec_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pick_windows(self, K: int) -> int:
        return int(lib().tdec_pick_windows(self._h, int(K)))

    def set_max_windows(self, max_nw: int):
        """Limit the window choice to at most max_nw per block (0: no limit)."""
        _check("tdec_set_max_windows", lib().tdec_set_max_windows(self._h, int(max_nw)))

    def cb_decode_batch(self, descs, llr, p: Params, bits=None, crc_ok=None, iters=None,
                        stream=None):
        """llr: int16 CUDA tensor; bits: uint8 CUDA tensor or None; crc_ok /
        iters: uint8 CUDA tensors with one entry per code block."""
        n = len(descs)
        n_llr, n_bits = _desc_extent(descs)
        _need(llr, "int16", n_llr, "llr")
        if bits is not None:
            _need(bits, "uint8", n_bits, "bits")
        _need(crc_ok, "uint8", n, "crc_ok")
        _need(iters, "uint8", n, "iters")
        _check("cb_decode_batch",
               lib().cb_decode_batch(self._h, n, ct.cast(descs, ct.c_void_p), _dptr(llr),
                                     ct.byref(p), _dptr(bits), _dptr(crc_ok), _dptr(iters),
                                     _stream(stream)))

    def cb_decode_batch_fixed(self, descs, llr, p: Params, bits=None, crc_ok=None, iters=None,
                              stream=None):
        """cb_decode_batch through the allocation-free entry point (the decode
        kernel's scratch is the library's fixed device array)."""
        n = len(descs)
        n_llr, n_bits = _desc_extent(descs)
        _need(llr, "int16", n_llr, "llr")
        if bits is not None:
            _need(bits, "uint8", n_bits, "bits")
        _need(crc_ok, "uint8", n, "crc_ok")
        _need(iters, "uint8", n, "iters")
        _check("cb_decode_batch_fixed",
               lib().cb_decode_batch_fixed(self._h, n, ct.cast(descs, ct.c_void_p), _dptr(llr),
                                           ct.byref(p), _dptr(bits), _dptr(crc_ok),
                                           _dptr(iters), _stream(stream)))

    def tb_decode(self, llr, tbs: int, p: Params, bits, res, stream=None):
        """res: uint8 CUDA tensor of TB_RESULT_BYTES bytes."""
        _need(llr, "int16", tb_llr_count(tbs), "llr")
        if bits is not None:
            _need(bits, "uint8", (tbs + 7) // 8, "bits")
        _need(res, "uint8", TB_RESULT_BYTES, "res")
        _check("tb_decode", lib().tb_decode(self._h, _dptr(llr), int(tbs), ct.byref(p),
                                            _dptr(bits), _dptr(res), _stream(stream)))

    def tb_decode_batch(self, tbs, llr_off, bits_off, llr, p: Params, bits, res, stream=None):
        tbs = np.ascontiguousarray(tbs, np.int32)
        llr_off = np.ascontiguousarray(llr_off, np.int64)
        bits_off = None if bits_off is None else np.ascontiguousarray(bits_off, np.int64)
        n = tbs.size
        if n:
            counts = np.array([tb_llr_count(int(t)) for t in tbs], np.int64)
            _need(llr, "int16", int((llr_off + counts).max()), "llr")
            if bits is not None:
                _need(bits, "uint8", int((bits_off + (tbs.astype(np.int64) + 7) // 8).max()), "bits")
        _need(res, "uint8", n * TB_RESULT_BYTES, "res")
        _check("tb_decode_batch",
               lib().tb_decode_batch(self._h, tbs.size, _np_ptr(tbs), _np_ptr(llr_off),
                                     _np_ptr(bits_off), _dptr(llr), ct.byref(p), _dptr(bits),
                                     _dptr(res), _stream(stream)))

    def graph_cb_decode(self, descs, llr, p: Params, bits=None, crc_ok=None, iters=None):
        """Plan and capture a code block batch; returns a Graph whose launch()
        replays it (the tensors must outlive the Graph)."""
        n_llr, n_bits = _desc_extent(descs)
        _need(llr, "int16", n_llr, "llr")
        if bits is not None:
            _need(bits, "uint8", n_bits, "bits")
        _need(crc_ok, "uint8", len(descs), "crc_ok")
        _need(iters, "uint8", len(descs), "iters")
        h = ct.c_void_p()
        _check("tdec_graph_cb_decode",
               lib().tdec_graph_cb_decode(self._h, len(descs), ct.cast(descs, ct.c_void_p),
                                          _dptr(llr), ct.byref(p), _dptr(bits), _dptr(crc_ok),
                                          _dptr(iters), ct.byref(h)))
        return Graph(h, self, (llr, bits, crc_ok, iters))

    def graph_tb_decode(self, tbs, llr_off, bits_off, llr, p: Params, bits, res):
        tbs = np.ascontiguousarray(tbs, np.int32)
        llr_off = np.ascontiguousarray(llr_off, np.int64)
        bits_off = None if bits_off is None else np.ascontiguousarray(bits_off, np.int64)
        counts = np.array([tb_llr_count(int(t)) for t in tbs], np.int64)
        _need(llr, "int16", int((llr_off + counts).max()), "llr")
        if bits is not None:
            _need(bits, "uint8", int((bits_off + (tbs.astype(np.int64) + 7) // 8).max()), "bits")
        _need(res, "uint8", tbs.size * TB_RESULT_BYTES, "res")
        h = ct.c_void_p()
        _check("tdec_graph_tb_decode",
               lib().tdec_graph_tb_decode(self._h, tbs.size, _np_ptr(tbs), _np_ptr(llr_off),
                                          _np_ptr(bits_off), _dptr(llr), ct.byref(p),
                                          _dptr(bits), _dptr(res), ct.byref(h)))
        return Graph(h, self, (llr, bits, res))

    def autotune(self, Ks, min_W=64, max_iters=6, batch_bits=25_000_000, stream=None):
        """Measure and set the window count of each size in Ks; returns
        {K: (n_windows, ns per 1000 code block bits)}."""
        Ks = np.ascontiguousarray(Ks, np.int32)
        nw = np.zeros(Ks.size, np.int32)
        ns = np.zeros(Ks.size, np.float32)
        _check("tdec_autotune",
               lib().tdec_autotune(self._h, Ks.size, _np_ptr(Ks), int(min_W), int(max_iters),
                                   int(batch_bits), _np_ptr(nw), _np_ptr(ns), _stream(stream)))
        return {int(k): (int(a), float(b)) for k, a, b in zip(Ks, nw, ns)}

    def autotune_reset(self):
        lib().tdec_autotune_reset(self._h)

    def set_knobs(self, lds_budget=30720, order=ORDER_K_DESC, win_target=0, grid_cap=0):
        k = Knobs(int(lds_budget), int(order), int(win_target), int(grid_cap), 0.0)
        _check("tdec_set_knobs", lib().tdec_set_knobs(self._h, ct.byref(k)))

    def get_knobs(self):
        k = Knobs()
        _check("tdec_get_knobs", lib().tdec_get_knobs(self._h, ct.byref(k)))
        return k.as_dict()

    def autotune_batch(self, tbs, llr_off, llr, p: Params, min_W=32, stream=None):
        """Measure the launch knobs on one batch of transport blocks and set
        the fastest; returns {"best", "rule", "candidates"} (knob dicts with
        their launch time "us")."""
        tbs = np.ascontiguousarray(tbs, np.int32)
        llr_off = np.ascontiguousarray(llr_off, np.int64)
        counts = np.array([tb_llr_count(int(t)) for t in tbs], np.int64)
        _need(llr, "int16", int((llr_off + counts).max()), "llr")
        cands = (Knobs * 256)()
        n = ct.c_int32()
        best, rule = Knobs(), Knobs()
        _check("tdec_autotune_batch",
               lib().tdec_autotune_batch(self._h, tbs.size, _np_ptr(tbs), _np_ptr(llr_off),
                                         _dptr(llr), ct.byref(p), int(min_W), cands, 256,
                                         ct.byref(n), ct.byref(best), ct.byref(rule),
                                         _stream(stream)))
        return {"best": best.as_dict(), "rule": rule.as_dict(),
                "candidates": [cands[i].as_dict() for i in range(n.value)]}

    def derate_batch(self, descs, e, soft, combine: int, stream=None):
        """e: int8 or int16 CUDA tensor of soft values; soft: int16 CUDA
        tensor of [3][K+4] soft buffers (HARQ state)."""
        if len(descs) == 0:
            return
        ne, ns = _rm_extent(descs)
        eb = {"torch.int8": 1, "torch.int16": 2}.get(str(e.dtype))
        if eb is None:
            raise ValueError("e: int8 or int16 tensor expected")
        _need(e, str(e.dtype)[6:], ne, "e")
        _need(soft, "int16", ns, "soft")
        _check("tdec_derate_batch",
               lib().tdec_derate_batch(self._h, len(descs), ct.cast(descs, ct.c_void_p), _dptr(e),
                                       eb, _dptr(soft), int(combine), _stream(stream)))

    def rate_match_batch(self, descs, coded, e, stream=None):
        if len(descs) == 0:
            return
        ne, nc = _rm_extent(descs)
        _need(coded, "uint8", nc, "coded")
        _need(e, "uint8", ne, "e")
        _check("tdec_rate_match_batch",
               lib().tdec_rate_match_batch(self._h, len(descs), ct.cast(descs, ct.c_void_p),
                                           _dptr(coded), _dptr(e), _stream(stream)))

    def cb_encode_batch(self, descs, payload, coded, stream=None):
        n_llr, n_bits = _desc_extent(descs)
        _need(payload, "uint8", n_bits, "payload")
        _need(coded, "uint8", n_llr, "coded")
        _check("cb_encode_batch",
               lib().cb_encode_batch(self._h, len(descs), ct.cast(descs, ct.c_void_p),
                                     _dptr(payload), _dptr(coded), _stream(stream)))

    def tb_encode(self, payload, tbs: int, coded, stream=None):
        _need(payload, "uint8", (tbs + 7) // 8, "payload")
        _need(coded, "uint8", tb_llr_count(tbs), "coded")
        _check("tb_encode", lib().tb_encode(self._h, _dptr(payload), int(tbs), _dptr(coded),
                                            _stream(stream)))


class Graph:
    """A captured decode (tdec_graph); launch() enqueues one replay."""

    def __init__(self, h, decoder, keep):
        self._h, self._decoder, self._keep = h, decoder, keep

    def launch(self, stream=None):
        _check("tdec_graph_launch", lib().tdec_graph_launch(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().tdec_graph_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def parse_tb_results(raw: np.ndarray) -> list[dict]:
    """Decode the bytes of tdec_tb_result entries copied back to the host."""
    arr = np.frombuffer(np.ascontiguousarray(raw).tobytes(), dtype=TB_RESULT_DTYPE)
    out = []
    for r in arr:
        C = int(r["C"])
        out.append({"tb_ok": int(r["tb_ok"]), "max_iters_used": int(r["max_iters_used"]),
                    "C": C, "cb_ok": [int(x) for x in r["cb_ok"][:C]],
                    "cb_iters": [int(x) for x in r["cb_iters"][:C]]})
    return out


# ----------------------------------------------------------------------------- serving loop
def now_ns() -> int:
    """CLOCK_MONOTONIC in ns, the serving loop's time base."""
    return int(lib().tdec_now_ns())


def server_cfg(params: Params, deadline_us=3000, slot_budget_bytes=0, max_batch_cb=0,
               mode=SERVE_CONTINUOUS, admission=ADMIT_BUDGET, model_lat_ns=0,
               model_ns_per_kbit=0, max_inflight=0, ring_idle_us=0) -> ServerCfg:
    return ServerCfg(slot_budget_bytes, deadline_us, max_batch_cb, mode, admission,
                     model_lat_ns, model_ns_per_kbit, params, max_inflight, ring_idle_us)


class Server:
    """The native serving loop (include/tdec_server.h).  Create with a
    Decoder (GPU executor) or with Server.model(...) (modelled executor, no
    device)."""

    def __init__(self, decoder: "Decoder | None", cfg: ServerCfg, _model=None):
        h = ct.c_void_p()
        if _model is None:
            _check("tdec_server_create",
                   lib().tdec_server_create(decoder._h, ct.byref(cfg), ct.byref(h)))
        else:
            _check("tdec_server_create_model",
                   lib().tdec_server_create_model(ct.byref(cfg), int(_model[0]),
                                                  int(_model[1]), ct.byref(h)))
        self._h = h
        self._decoder = decoder  # keeps the context alive
        self._keep = {}          # tag -> buffers that must outlive the request

    @classmethod
    def model(cls, cfg: ServerCfg, lat_ns: int, ns_per_kbit: int) -> "Server":
        return cls(None, cfg, _model=(lat_ns, ns_per_kbit))

    def submit(self, tags, tbs, llr_ptrs, bits_ptrs=None, t_arrive_ns=None, keep=None,
               device=False):
        """Submit one arrival batch.  llr_ptrs / bits_ptrs: addresses (ints)
        of each block's int16 LLRs (host memory, or device memory with
        device=True) and payload buffer (host); `keep` (a list per block,
        optional) holds objects that must stay alive until the result is
        polled.  Returns (admitted count, status array)."""
        tags = np.ascontiguousarray(tags, np.uint64)
        tbs = np.ascontiguousarray(tbs, np.int32)
        n = tags.size
        if tbs.size != n or len(llr_ptrs) != n:
            raise ValueError("tags, tbs and llr_ptrs differ in length")
        lp = np.ascontiguousarray(llr_ptrs, np.uint64)
        bp = None if bits_ptrs is None else np.ascontiguousarray(bits_ptrs, np.uint64)
        st = np.zeros(n, np.int32)
        t = now_ns() if t_arrive_ns is None else int(t_arrive_ns)
        if keep is not None:
            for i in range(n):
                self._keep[int(tags[i])] = keep[i]
        fn = lib().tdec_server_submit_dev if device else lib().tdec_server_submit
        k = fn(self._h, n, _np_ptr(tags), _np_ptr(tbs), _np_ptr(lp), _np_ptr(bp), t, _np_ptr(st))
        if k < 0:
            raise TdecError("tdec_server_submit", k)
        return k, st

    def replay(self, counts, tbs, llr_ptrs, bits_ptrs=None, period_ns=1_000_000,
               t_first_ns=None, tag_base=0):
        """Submit a precomputed schedule from a native loop (device LLRs):
        counts[k] arrivals at tick k, tbs / llr_ptrs / bits_ptrs one entry
        per arrival.  Returns (max lateness of a tick, longest submit) in ns."""
        counts = np.ascontiguousarray(counts, np.int32)
        tbs = np.ascontiguousarray(tbs, np.int32)
        lp = np.ascontiguousarray(llr_ptrs, np.uint64)
        n = int(counts.sum())
        if tbs.size != n or lp.size != n:
            raise ValueError("tbs and llr_ptrs need one entry per arrival")
        bp = None if bits_ptrs is None else np.ascontiguousarray(bits_ptrs, np.uint64)
        if bp is not None and bp.size != n:
            raise ValueError("bits_ptrs needs one entry per arrival")
        late, smax = ct.c_int64(), ct.c_int64()
        t = now_ns() + period_ns if t_first_ns is None else int(t_first_ns)
        _check("tdec_server_replay",
               lib().tdec_server_replay(self._h, counts.size, t, int(period_ns), _np_ptr(counts),
                                        _np_ptr(tbs), _np_ptr(lp), _np_ptr(bp), int(tag_base),
                                        ct.byref(late), ct.byref(smax)))
        return late.value, smax.value

    def poll(self, max_n=4096, wait_us=0) -> list[dict]:
        buf = (ServeResult * max_n)()
        k = lib().tdec_server_poll(self._h, ct.cast(buf, ct.c_void_p), max_n, int(wait_us))
        out = []
        for r in buf[:k]:
            d = {n: getattr(r, n) for n, _ in ServeResult._fields_}
            self._keep.pop(int(r.tag), None)
            out.append(d)
        return out

    def discard(self, max_n=65536, wait_us=0) -> int:
        """Drop up to max_n finished results without converting them (for
        load generators that read the statistics only); returns the count.
        Buffers passed with `keep` stay referenced."""
        if getattr(self, "_rawbuf", None) is None or len(self._rawbuf) < max_n:
            self._rawbuf = (ServeResult * max_n)()
        return int(lib().tdec_server_poll(self._h, ct.cast(self._rawbuf, ct.c_void_p), max_n,
                                          int(wait_us)))

    def poll_array(self, max_n=65536, wait_us=0) -> np.ndarray:
        """Up to max_n finished results as a numpy structured array (fields of
        tdec_server_result), without a Python object per result (for load
        generators that keep a clock).  Buffers passed with `keep` stay
        referenced, as with discard()."""
        if getattr(self, "_rawbuf", None) is None or len(self._rawbuf) < max_n:
            self._rawbuf = (ServeResult * max_n)()
        k = int(lib().tdec_server_poll(self._h, ct.cast(self._rawbuf, ct.c_void_p), max_n,
                                       int(wait_us)))
        return np.ctypeslib.as_array(self._rawbuf)[:k].copy()

    def launches(self, max_n=4096) -> list[dict]:
        """Records of the most recent launches, oldest first (the server
        keeps the last 4096)."""
        buf = (LaunchRec * max_n)()
        k = lib().tdec_server_launches(self._h, ct.cast(buf, ct.c_void_p), max_n)
        if k < 0:
            raise TdecError("tdec_server_launches", k)
        return [{n: getattr(r, n) for n, _ in LaunchRec._fields_} for r in buf[:k]]

    def drain(self, timeout_ms=60000):
        _check("tdec_server_drain", lib().tdec_server_drain(self._h, int(timeout_ms)))

    def stats(self) -> dict:
        s = ServeStats()
        _check("tdec_server_stats", lib().tdec_server_stats(self._h, ct.byref(s)))
        return s.as_dict()

    def reset_stats(self):
        lib().tdec_server_reset_stats(self._h)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().tdec_server_destroy(self._h)
            self._h = ct.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
