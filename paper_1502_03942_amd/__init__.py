"""MI355X-native unsorted top-k selection (sampling method of Hübschle-Schneider,
Sanders, Müller, "Communication Efficient Algorithms for Top-k Selection
Problems", §2 Algorithm "communication efficient selection" and §4.1).

Thin ctypes binding over ``libtopk.so`` (declared in ``include/topk.h``): it
only marshals torch tensors into pointers, sizes and the current HIP stream.
Every step of the selection runs in the library's HIP kernels; there is no CPU
fallback -- a missing library raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtopk.so")

TOPK_LARGEST = 1
TOPK_SORTED = 2
TOPK_WRITE_KEYS = 4
TOPK_TRACE = 8
TOPK_GRAPH = 16
STATUS_OK = 0
STATUS_INTERNAL = 1
STATUS_BAD_ROW = 2
STATUS_BAD_KEY = 4
STATUS_SUM_RANGE = 8
STATUS_BAD_ARG = 16
ROUND_EXACT = -2

_lib = None


class RoundRecord(ctypes.Structure):
    _fields_ = [
        ("n_cur", ctypes.c_uint32), ("k_cur", ctypes.c_uint32),
        ("s", ctypes.c_uint32), ("c_num", ctypes.c_uint32),
        ("lo", ctypes.c_int64), ("hi", ctypes.c_int64),
        ("l_idx", ctypes.c_uint32), ("r_idx", ctypes.c_uint32),
        ("has_l", ctypes.c_uint32), ("has_r", ctypes.c_uint32),
        ("na", ctypes.c_uint32), ("nb", ctypes.c_uint32),
        ("ok", ctypes.c_uint32), ("tag", ctypes.c_uint32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TopkError(RuntimeError):
    pass


def lib():
    """Load libtopk.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise TopkError("libtopk.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, u32, i32, sz = (ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                             ctypes.c_int, ctypes.c_size_t)
    L.topk_create.argtypes = [ctypes.POINTER(vp), i32, u64]
    L.topk_destroy.argtypes = [vp]
    L.topk_destroy.restype = None
    L.topk_set_param.argtypes = [vp, ctypes.c_char_p, ctypes.c_int64]
    L.topk_get_param.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)]
    L.topk_workspace_bytes.argtypes = [vp, u64, u32]
    L.topk_workspace_bytes.restype = sz
    sel = [vp, vp, u64, u64, u32, vp, vp, vp, vp, vp, vp, sz, vp]
    L.topk_select_u32.argtypes = sel
    L.topk_select_f32.argtypes = sel
    L.topk_trace_rounds.argtypes = [vp, vp, u64, ctypes.POINTER(RoundRecord), u32,
                                    ctypes.POINTER(u32), vp]
    L.topk_trace_sample.argtypes = [vp, vp, u64, u32, vp, u32, ctypes.POINTER(u32), vp]
    L.topk_kernel_times.argtypes = [vp, vp, vp, u32, ctypes.POINTER(u32)]
    L.topk_batched_workspace_bytes.argtypes = [vp, u32, u32]
    L.topk_batched_workspace_bytes.restype = sz
    L.topk_select_batched_f32.argtypes = [vp, vp, vp, u32, vp, vp, u32, vp, vp, vp, vp, vp, sz, vp]
    L.topk_select_batched_f32_noalloc.argtypes = [vp, vp, vp, u32, vp, vp, u32, vp, vp, vp, vp, vp]
    L.topk_tune_batched_f32.argtypes = [vp, vp, vp, u32, vp, vp, u32, vp, vp, vp, vp, vp, sz, u32, vp]
    L.topk_save_tuning.argtypes = [vp, ctypes.c_char_p]
    L.topk_tune_f32.argtypes = [vp, vp, ctypes.c_uint64, ctypes.c_uint64, u32, vp, vp, vp, vp, sz,
                                u32, vp]
    L.topk_stream_read.argtypes = [vp, vp, ctypes.c_uint64, vp, vp]
    L.topk_load_tuning.argtypes = [vp, ctypes.c_char_p]
    L.topk_rows_fwd_f32.argtypes = [vp, vp, u32, u32, u32, u32, vp, vp, vp]
    L.topk_scatter_bwd_f32.argtypes = [vp, vp, u32, u32, u32, vp, vp]
    L.topk_frequent_workspace_bytes.argtypes = [vp, u64, u32]
    L.topk_frequent_workspace_bytes.restype = sz
    L.topk_frequent_u32.argtypes = [vp, vp, u64, u32, u32, u32, u64, vp, vp, vp, vp, vp, vp, sz, vp]
    L.topk_sum_workspace_bytes.argtypes = [vp, u64, u32]
    L.topk_sum_workspace_bytes.restype = sz
    L.topk_sum_top_u32.argtypes = [vp, vp, vp, u64, u32, u32, u32, u64, vp, vp, vp, vp, vp, vp,
                                   sz, vp]
    L.topk_sample_size.argtypes = [i32, u64, u32, u32, ctypes.c_double, ctypes.c_double]
    L.topk_sample_size.restype = ctypes.c_double
    L.topk_sample_threshold.argtypes = [u64, ctypes.c_double]
    L.topk_sample_threshold.restype = u64
    ms = [vp, vp, vp, u32, u64, u32, vp, vp, vp, vp, vp, vp]
    L.topk_msselect_u32.argtypes = ms
    L.topk_msselect_f32.argtypes = ms
    ams = [vp, vp, vp, u32, u64, u64, u32, vp, vp, vp, vp, vp]
    L.topk_amsselect_u32.argtypes = ams
    L.topk_amsselect_f32.argtypes = ams
    L.topk_strerror.argtypes = [i32]
    L.topk_strerror.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise TopkError("libtopk: %s (%d)" % (lib().topk_strerror(rc).decode(), rc))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """A libtopk context on one device: tuning parameters and the sampler seed."""

    def __init__(self, device=0, seed=0x5EED):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        h = ctypes.c_void_p()
        _check(lib().topk_create(ctypes.byref(h), self.device.index or 0, seed))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.topk_destroy(h)
            self._h = None

    def set_param(self, name, value):
        _check(lib().topk_set_param(self._h, name.encode(), int(value)))
        return self

    def get_param(self, name):
        v = ctypes.c_int64()
        _check(lib().topk_get_param(self._h, name.encode(), ctypes.byref(v)))
        return v.value

    def workspace_bytes(self, n, flags=0):
        return int(lib().topk_workspace_bytes(self._h, n, flags))

    def workspace(self, n, flags=0):
        return torch.empty(max(self.workspace_bytes(n, flags), 256), dtype=torch.uint8,
                           device=self.device)

    def select(self, keys, k, largest=False, write_keys=False, trace=False, workspace=None,
               sorted=False):
        """Select the k smallest (or largest) of a 1-D u32/f32 CUDA tensor.

        u32 keys are passed as torch.uint32 or as torch.int32 holding the bits.
        Returns a dict of device tensors: ``idx`` (int32 holding u32 positions,
        length k, in an unspecified order, or with ``sorted`` in the order by
        (key, position)), ``kth_key`` (1 element, dtype of keys), ``kth_idx``,
        ``status`` and, with ``write_keys``, ``keys``.  ``workspace`` is kept
        in the dict for trace queries.
        """
        if keys.dim() != 1 or not keys.is_cuda:
            raise ValueError("keys must be a 1-D CUDA tensor")
        if keys.dtype == torch.float32:
            fn, is_f32 = lib().topk_select_f32, True
        elif keys.dtype in (torch.int32, torch.uint32):
            fn, is_f32 = lib().topk_select_u32, False
        else:
            raise TypeError("keys must be float32 or uint32/int32 bits")
        n = keys.numel()
        flags = (TOPK_LARGEST if largest else 0) | (TOPK_WRITE_KEYS if write_keys else 0) | \
                (TOPK_TRACE if trace else 0) | (TOPK_SORTED if sorted else 0)
        dev = keys.device
        out_idx = torch.empty(max(k, 1), dtype=torch.int32, device=dev)
        kth_key = torch.empty(1, dtype=keys.dtype, device=dev)
        kth_idx = torch.empty(1, dtype=torch.int32, device=dev)
        status = torch.empty(1, dtype=torch.int32, device=dev)     # every call writes it
        out_keys = torch.empty(max(k, 1), dtype=keys.dtype, device=dev) if write_keys else None
        if workspace is None:
            workspace = self.workspace(n, flags)
        _check(fn(self._h, _ptr(keys), n, k, flags, _ptr(out_idx), _ptr(out_keys),
                  _ptr(kth_key), _ptr(kth_idx), _ptr(status), _ptr(workspace),
                  workspace.numel(), _stream(dev)))
        res = {"idx": out_idx[:k], "kth_key": kth_key, "kth_idx": kth_idx,
               "status": status, "workspace": workspace, "n": n}
        if write_keys:
            res["keys"] = out_keys[:k]
        return res

    def tune(self, keys, k, largest=False, reps=3, workspace=None):
        """Autotune s_target and c_num for this selection (topk_tune_f32, f32
        keys); returns the output dict of a call with the chosen parameters."""
        if keys.dtype != torch.float32 or keys.dim() != 1 or not keys.is_cuda:
            raise TypeError("tune: keys must be a 1-D float32 CUDA tensor")
        n = keys.numel()
        flags = TOPK_LARGEST if largest else 0
        if workspace is None:
            workspace = self.workspace(n, flags)
        dev = keys.device
        out_idx = torch.empty(max(k, 1), dtype=torch.int32, device=dev)
        kth_key = torch.empty(1, dtype=torch.float32, device=dev)
        kth_idx = torch.empty(1, dtype=torch.int32, device=dev)
        _check(lib().topk_tune_f32(self._h, _ptr(keys), n, k, flags, _ptr(out_idx), _ptr(kth_key),
                                   _ptr(kth_idx), _ptr(workspace), workspace.numel(), int(reps),
                                   _stream(dev)))
        return self.select(keys, k, largest=largest, workspace=workspace)

    def stream_read(self, keys, sink):
        """One plain read of keys (1-D, 4-byte elements, numel a multiple of
        4096) with the first sweep's access pattern (topk_stream_read): a
        bandwidth reference, not a selection."""
        _check(lib().topk_stream_read(self._h, _ptr(keys), keys.numel(), _ptr(sink),
                                      _stream(keys.device)))

    KERNEL_KINDS = ("pivot_first", "pivot", "sweep_first", "sweep", "tail")

    def batched_workspace(self, rows, flags=0):
        nb = int(lib().topk_batched_workspace_bytes(self._h, rows, flags))
        return torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)

    def select_batched(self, keys, row_off, k, out_off=None, largest=False, graph=False,
                       workspace=None, out=None):
        """Per-row top-k of a CSR batch (topk_select_batched_f32).

        keys f32 [sum len], row_off int64 [R+1], k int32 [R] (all CUDA); out_off
        int64 [R+1] (exclusive prefix of k) is computed on the device if None.
        Returns a dict: ``idx`` (int32 holding u32 columns, length sum k),
        ``kth_key`` f32 [R], ``kth_idx`` (int32 holding u32) [R], ``status``,
        ``out_off``.  ``out`` (a dict from an earlier call with the same shapes)
        reuses its buffers, which keeps a captured graph valid.
        """
        R = row_off.numel() - 1
        if keys.dtype != torch.float32 or keys.dim() != 1 or not keys.is_cuda:
            raise TopkError("select_batched: keys must be a 1-D float32 CUDA tensor")
        if row_off.dtype not in (torch.int64, torch.uint64) or k.dtype not in (torch.int32, torch.uint32):
            raise TopkError("select_batched: row_off int64 [R+1] and k int32 [R] expected")
        if out is None:
            if out_off is None:
                out_off = torch.zeros(R + 1, dtype=torch.int64, device=keys.device)
                out_off[1:] = torch.cumsum(k.to(torch.int64), 0)
            total = int(out_off[-1].item())
            out = {"idx": torch.empty(max(total, 1), dtype=torch.int32, device=keys.device),
                   "kth_key": torch.empty(R, dtype=torch.float32, device=keys.device),
                   "kth_idx": torch.empty(R, dtype=torch.int32, device=keys.device),
                   "status": torch.zeros(1, dtype=torch.int32, device=keys.device),
                   "out_off": out_off}
        ws = workspace if workspace is not None else out.get("workspace")
        if ws is None:
            ws = self.batched_workspace(R)
        out["workspace"] = ws
        flags = (TOPK_LARGEST if largest else 0) | (TOPK_GRAPH if graph else 0)
        _check(lib().topk_select_batched_f32(
            self._h, _ptr(keys), _ptr(row_off), R, _ptr(k), _ptr(out["out_off"]), flags,
            _ptr(out["idx"]), _ptr(out["kth_key"]), _ptr(out["kth_idx"]), _ptr(out["status"]),
            _ptr(ws), ws.numel(), _stream(keys.device)))
        return out

    def select_batched_noalloc(self, keys, row_off, k, out_off, out, largest=False):
        """topk_select_batched_f32_noalloc: the batched selection with the
        library's static scratch instead of a workspace.  ``out`` is a dict of
        caller-allocated outputs (``idx``, ``kth_key``, ``kth_idx``,
        ``status``); nothing is allocated here."""
        R = row_off.numel() - 1
        _check(lib().topk_select_batched_f32_noalloc(
            self._h, _ptr(keys), _ptr(row_off), R, _ptr(k), _ptr(out_off),
            TOPK_LARGEST if largest else 0, _ptr(out["idx"]), _ptr(out["kth_key"]),
            _ptr(out["kth_idx"]), _ptr(out["status"]), _stream(keys.device)))
        return out

    def tune_batched(self, keys, row_off, k, out_off=None, largest=False, reps=3, out=None):
        """Autotune the batched form on this batch (topk_tune_batched_f32);
        returns the output dict of the last timed call (valid results)."""
        out = self.select_batched(keys, row_off, k, out_off=out_off, largest=largest, out=out)
        R = row_off.numel() - 1
        ws = out["workspace"]
        _check(lib().topk_tune_batched_f32(
            self._h, _ptr(keys), _ptr(row_off), R, _ptr(k), _ptr(out["out_off"]),
            TOPK_LARGEST if largest else 0, _ptr(out["idx"]), _ptr(out["kth_key"]),
            _ptr(out["kth_idx"]), _ptr(out["status"]), _ptr(ws), ws.numel(), int(reps),
            _stream(keys.device)))
        return out

    def save_tuning(self, path):
        _check(lib().topk_save_tuning(self._h, os.fsencode(path)))

    def load_tuning(self, path=None):
        _check(lib().topk_load_tuning(self._h, None if path is None else os.fsencode(path)))
        return self

    def kernel_times(self, max_records=1 << 16):
        """Durations (ms) of the kernels recorded with param "timing" > 0 since
        the last read-out, as a list of (kind, ms) in enqueue order."""
        ms = (ctypes.c_float * max_records)()
        kind = (ctypes.c_int32 * max_records)()
        cnt = ctypes.c_uint32()
        _check(lib().topk_kernel_times(self._h, ms, kind, max_records, ctypes.byref(cnt)))
        return [(self.KERNEL_KINDS[kind[i]], ms[i]) for i in range(min(cnt.value, max_records))]

    def trace_rounds(self, res):
        """Round records of the call that returned ``res`` (topk_trace_rounds)."""
        cap = 64
        recs = (RoundRecord * cap)()
        cnt = ctypes.c_uint32()
        _check(lib().topk_trace_rounds(self._h, _ptr(res["workspace"]), res["n"], recs, cap,
                                       ctypes.byref(cnt), _stream(res["workspace"].device)))
        return [recs[i].as_dict() for i in range(min(cnt.value, cap))]

    def trace_sample(self, res, tag):
        """Sampled objects (input positions, unordered) of attempt ``tag`` of the
        call that returned ``res``, made with ``trace=True`` (topk_trace_sample)."""
        cap = 1 << 16
        buf = (ctypes.c_uint32 * cap)()
        cnt = ctypes.c_uint32()
        _check(lib().topk_trace_sample(self._h, _ptr(res["workspace"]), res["n"], tag, buf, cap,
                                       ctypes.byref(cnt), _stream(res["workspace"].device)))
        return list(buf[:min(cnt.value, cap)])


    # ---- top-k most frequent objects (§7) and top-k sum aggregation (§8) ----

    def frequent(self, keys, U, k, kstar=0, T=1 << 32, tables=False, workspace=None):
        """The k most frequent objects of a 1-D int32/uint32 CUDA tensor of
        objects in [0, U) (topk_frequent_u32): PAC when kstar = 0, else EC
        counting kstar candidates exactly; sampling rate T / 2^32.

        Returns a dict of device tensors: ``ids`` [k] and ``counts`` [k] (most
        frequent first; PAC: sample counts, EC: exact counts), ``status`` and,
        with ``tables``, ``sample_counts`` [U] and ``n_sampled`` [1]."""
        if keys.dim() != 1 or not keys.is_cuda or keys.dtype not in (torch.int32, torch.uint32):
            raise TopkError("frequent: keys must be a 1-D int32/uint32 CUDA tensor")
        dev = keys.device
        n = keys.numel()
        if workspace is None:
            nb = int(lib().topk_frequent_workspace_bytes(self._h, n, U))
            workspace = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
        out = {"ids": torch.empty(k, dtype=torch.int32, device=dev),
               "counts": torch.empty(k, dtype=torch.int32, device=dev),
               "status": torch.empty(1, dtype=torch.int32, device=dev)}
        if tables:
            out["sample_counts"] = torch.empty(U, dtype=torch.int32, device=dev)
            out["n_sampled"] = torch.empty(1, dtype=torch.int64, device=dev)
        _check(lib().topk_frequent_u32(
            self._h, _ptr(keys), n, U, k, kstar, int(T), _ptr(out["ids"]), _ptr(out["counts"]),
            _ptr(out.get("sample_counts")), _ptr(out.get("n_sampled")), _ptr(out["status"]),
            _ptr(workspace), workspace.numel(), _stream(dev)))
        return out

    def sum_top(self, keys, values, U, k, s, kstar=0, tables=False, workspace=None):
        """The k keys with the largest sums of values (topk_sum_top_u32): the
        input aggregated by key, a weighted sample of size about s, then PAC
        (kstar = 0, values = sample counts) or the kstar most sampled keys
        ranked by exact sum.  keys/values: 1-D int32/uint32 CUDA tensors.

        Returns ``ids`` [k], ``vals`` [k] (int64), ``status`` and, with
        ``tables``, ``sums`` [U] (int64) and ``samples`` [U]."""
        for t in (keys, values):
            if t.dim() != 1 or not t.is_cuda or t.dtype not in (torch.int32, torch.uint32):
                raise TopkError("sum_top: keys and values must be 1-D int32/uint32 CUDA tensors")
        dev = keys.device
        n = keys.numel()
        if workspace is None:
            nb = int(lib().topk_sum_workspace_bytes(self._h, n, U))
            workspace = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
        out = {"ids": torch.empty(k, dtype=torch.int32, device=dev),
               "vals": torch.empty(k, dtype=torch.int64, device=dev),
               "status": torch.empty(1, dtype=torch.int32, device=dev)}
        if tables:
            out["sums"] = torch.empty(U, dtype=torch.int64, device=dev)
            out["samples"] = torch.empty(U, dtype=torch.int32, device=dev)
        _check(lib().topk_sum_top_u32(
            self._h, _ptr(keys), _ptr(values), n, U, k, kstar, int(s), _ptr(out["ids"]),
            _ptr(out["vals"]), _ptr(out.get("sums")), _ptr(out.get("samples")),
            _ptr(out["status"]), _ptr(workspace), workspace.numel(), _stream(dev)))
        return out


    # ---- selection over sorted rows: msSelect (App. A), amsSelect (§4.3) ----

    def _ms_keys(self, keys, row_off):
        if keys.dim() != 1 or not keys.is_cuda:
            raise TopkError("keys must be a 1-D CUDA tensor")
        if row_off.dtype not in (torch.int64, torch.uint64) or not row_off.is_cuda:
            raise TopkError("row_off must be an int64 CUDA tensor [p + 1]")
        if keys.dtype == torch.float32:
            return True
        if keys.dtype in (torch.int32, torch.uint32):
            return False
        raise TopkError("keys must be float32 or uint32/int32 bits")

    def msselect(self, keys, row_off, k, largest=False):
        """The object of rank k among sorted rows (topk_msselect_*): rows of a
        CSR batch, each sorted in the selection order.  Returns device tensors
        ``split`` [p] (selected prefix length per row), ``kth_pos``,
        ``kth_key``, ``rounds``, ``status``."""
        f32 = self._ms_keys(keys, row_off)
        p = row_off.numel() - 1
        dev = keys.device
        out = {"split": torch.empty(p, dtype=torch.int32, device=dev),
               "kth_pos": torch.empty(1, dtype=torch.int32, device=dev),
               "kth_key": torch.empty(1, dtype=keys.dtype, device=dev),
               "rounds": torch.zeros(1, dtype=torch.int32, device=dev),
               "status": torch.empty(1, dtype=torch.int32, device=dev)}
        fn = lib().topk_msselect_f32 if f32 else lib().topk_msselect_u32
        _check(fn(self._h, _ptr(keys), _ptr(row_off), p, int(k), TOPK_LARGEST if largest else 0,
                  _ptr(out["split"]), _ptr(out["kth_pos"]), _ptr(out["kth_key"]),
                  _ptr(out["rounds"]), _ptr(out["status"]), _stream(dev)))
        return out

    def amsselect(self, keys, row_off, kmin, kmax, largest=False):
        """The k smallest objects of sorted rows for some k in [kmin, kmax]
        (topk_amsselect_*).  Returns ``split`` [p], ``k`` (the k chosen),
        ``rounds``, ``status``."""
        f32 = self._ms_keys(keys, row_off)
        p = row_off.numel() - 1
        dev = keys.device
        out = {"split": torch.empty(p, dtype=torch.int32, device=dev),
               "k": torch.empty(1, dtype=torch.int64, device=dev),
               "rounds": torch.zeros(1, dtype=torch.int32, device=dev),
               "status": torch.empty(1, dtype=torch.int32, device=dev)}
        fn = lib().topk_amsselect_f32 if f32 else lib().topk_amsselect_u32
        _check(fn(self._h, _ptr(keys), _ptr(row_off), p, int(kmin), int(kmax),
                  TOPK_LARGEST if largest else 0, _ptr(out["split"]), _ptr(out["k"]),
                  _ptr(out["rounds"]), _ptr(out["status"]), _stream(dev)))
        return out


SAMPLE_PAC, SAMPLE_EC, SAMPLE_SUM = 0, 1, 2


def sample_size(method, n, k=0, kstar=0, eps=1e-3, delta=1e-3):
    """Expected sample size of §7 / §8 for an (eps, delta)-approximation
    (topk_sample_size: SAMPLE_PAC, SAMPLE_EC or SAMPLE_SUM)."""
    return float(lib().topk_sample_size(method, n, k, kstar, eps, delta))


def sample_threshold(n, size):
    """T = min(2^32, ceil(size 2^32 / n)): the sampling rate as a threshold."""
    return int(lib().topk_sample_threshold(n, float(size)))


_default = {}


def default_context(device=None):
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    key = dev.index or 0
    if key not in _default:
        _default[key] = Context(key)
    return _default[key]


def select(keys, k, largest=False, write_keys=False):
    """Top-k selection of a 1-D CUDA tensor with the device's default context."""
    return default_context(keys.device).select(keys, k, largest=largest, write_keys=write_keys)


# ---------------------------------------------------------------------------
# Row-wise top-k and its gradient (a differentiable layer).
# ---------------------------------------------------------------------------
def rows_fwd(scores, k, largest=True):
    """Row-wise top-k of a 2-D f32 CUDA tensor (topk_rows_fwd_f32).

    Returns (values f32 [B, k], indices int64 [B, k]) in selection order:
    values descending with ties by ascending column when ``largest``.
    """
    if scores.dim() != 2 or not scores.is_cuda or scores.dtype != torch.float32:
        raise TopkError("rows_fwd: scores must be a 2-D float32 CUDA tensor")
    scores = scores.contiguous()
    B, N = scores.shape
    values = torch.empty((B, k), dtype=torch.float32, device=scores.device)
    indices = torch.empty((B, k), dtype=torch.int64, device=scores.device)
    _check(lib().topk_rows_fwd_f32(None, _ptr(scores), B, N, k, TOPK_LARGEST if largest else 0,
                                   _ptr(values), _ptr(indices), _stream(scores.device)))
    return values, indices


def scatter_bwd(grad_out, indices, n_cols):
    """Dense gradient of row-wise top-k values (topk_scatter_bwd_f32)."""
    if grad_out.dim() != 2 or grad_out.dtype != torch.float32 or indices.dtype != torch.int64:
        raise TopkError("scatter_bwd: grad_out f32 [B, k] and indices int64 [B, k] expected")
    grad_out = grad_out.contiguous()
    indices = indices.contiguous()
    B, k = grad_out.shape
    grad_in = torch.empty((B, n_cols), dtype=torch.float32, device=grad_out.device)
    _check(lib().topk_scatter_bwd_f32(_ptr(grad_out), _ptr(indices), B, n_cols, k,
                                      _ptr(grad_in), _stream(grad_out.device)))
    return grad_in


class TopK(torch.autograd.Function):
    """values, indices = TopK.apply(scores, k, largest): row-wise top-k whose
    backward scatters the values' gradient back to the selected columns."""

    @staticmethod
    def forward(ctx, scores, k, largest=True):
        values, indices = rows_fwd(scores, k, largest)
        ctx.save_for_backward(indices)
        ctx.n_cols = scores.shape[1]
        ctx.mark_non_differentiable(indices)
        return values, indices

    @staticmethod
    def backward(ctx, grad_values, grad_indices):
        (indices,) = ctx.saved_tensors
        return scatter_bwd(grad_values, indices, ctx.n_cols), None, None


def topk(scores, k, largest=True):
    """Differentiable row-wise top-k: (values, indices), like torch.topk(scores, k, dim=1)."""
    return TopK.apply(scores, k, largest)
