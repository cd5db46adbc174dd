"""CPU model of the single-instance round policy (ctypes over topk_model.c).

TEST INFRASTRUCTURE ONLY, distinct from the oracle: the oracle defines the
result, this model mirrors the implementation's sampling and retry choices so
that the device's round trace can be compared with a CPU run of the same
policy.  Built with gcc on first use.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "topk_model.c")
LIB = os.path.join(_HERE, "libtopkmodel.so")
ROUND_EXACT = -2
_lib = None


class Round(ctypes.Structure):
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


class Params(ctypes.Structure):
    _fields_ = [
        ("s_target", ctypes.c_uint32), ("c_num", ctypes.c_uint32),
        ("nseg", ctypes.c_uint32), ("seg_cap", ctypes.c_uint32),
        ("t_fin", ctypes.c_uint32), ("r_max", ctypes.c_uint32),
        ("band_cap", ctypes.c_uint64), ("seed", ctypes.c_uint64),
        ("s_max", ctypes.c_uint32), ("pad", ctypes.c_uint32),
    ]


def build():
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        L.mdl_replay.argtypes = [vp, i32, u64, u64, i32, ctypes.POINTER(Params), vp, vp,
                                 ctypes.POINTER(Round), u32, vp]
        L.mdl_hash_taken.argtypes = [u64, u32, u32, u64]
        L.mdl_band_threshold.argtypes = [u64, u64, ctypes.c_int64, ctypes.c_int64, u64]
        L.mdl_band_threshold.restype = u64
        _lib = L
    return _lib


def _keys(keys):
    keys = np.ascontiguousarray(keys)
    if keys.dtype == np.float32:
        return keys, 1
    if keys.dtype == np.uint32:
        return keys, 0
    raise TypeError(keys.dtype)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def replay(keys, k, largest=False, *, s_target, c_num, nseg, seg_cap, t_fin, r_max,
           band_cap, seed, s_max=16384, max_recs=64):
    """Run the device's round policy on the CPU.

    Returns (status, out_idx[k] in the order the rounds write them, kth_idx,
    list of per-round dicts)."""
    keys, f = _keys(keys)
    prm = Params(s_target, c_num, nseg, seg_cap, t_fin, r_max, band_cap, seed, s_max, 0)
    out = np.zeros(k, np.uint32)
    kth = np.zeros(1, np.uint32)
    recs = (Round * max_recs)()
    nrec = np.zeros(1, np.uint32)
    rc = lib().mdl_replay(_p(keys), f, keys.size, k, int(largest), ctypes.byref(prm),
                          _p(out), _p(kth), recs, max_recs, _p(nrec))
    n = min(int(nrec[0]), max_recs)
    return rc, out, int(kth[0]), [recs[i].as_dict() for i in range(n)]


def hash_taken(seed, tag, x, T):
    return bool(lib().mdl_hash_taken(seed, tag, x, T))


def band_threshold(n_cur, s, lo, hi, s_target):
    return int(lib().mdl_band_threshold(n_cur, s, lo, hi, s_target))
