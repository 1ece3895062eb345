"""ctypes declarations of libljmd (include/ljmd.h).

Loads paper_2508_13523_amd/lib/libljmd.so, built by build.py.  There is no
fallback: if the library is missing, loading raises, so nothing can silently
run elsewhere.
"""
import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libljmd.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ljmd.h")

MAX_TYPES = 4
STATUS_WORDS = 4

OK = 0
EINVAL = -1
EBOX = -2
EWORKSPACE = -3
ENEIGH_OVERFLOW = -4
ENOTSUP = -5
EHIP = -6
ESCRATCH = -7
NOALLOC_MAX_BLOCKS = 16384

PREC_FP64 = 0
PREC_MIXED = 1 << 0
EV = 1 << 1
SYNC_CHECK = 1 << 2
SETUP = 1 << 3
SORT = 1 << 4
SEPARATE_KICK = 1 << 5
TUNE_TILES = 1 << 6
TUNE_MD = 1 << 7

FULL = 0
HALF = 1

FMT_GLOBAL = 0
FMT_TILED = 1
NL_GLOBAL = 1
NL_SORTED = 2
NL_BATCH = 4

ST_OVERFLOW, ST_NEED, ST_DANGEROUS, ST_NONFINITE = range(4)


class Box(ctypes.Structure):
    _fields_ = [("len", ctypes.c_double * 3)]


class Params(ctypes.Structure):
    _fields_ = [
        ("ntypes", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("eps", (ctypes.c_double * MAX_TYPES) * MAX_TYPES),
        ("sigma", (ctypes.c_double * MAX_TYPES) * MAX_TYPES),
        ("rc", (ctypes.c_double * MAX_TYPES) * MAX_TYPES),
        ("skin", ctypes.c_double),
        ("mass", ctypes.c_double * MAX_TYPES),
    ]


class NList(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("mode", ctypes.c_int32),
        ("cap", ctypes.c_int32),
        ("numneigh", ctypes.c_void_p),
        ("neigh", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
        ("xref", ctypes.c_void_p),
        ("aux", ctypes.c_void_p),
        ("aux_bytes", ctypes.c_size_t),
        ("flags", ctypes.c_int32),
        ("format", ctypes.c_int32),
        ("tile", ctypes.c_int32 * 3),
        ("ncell", ctypes.c_int32 * 3),
    ]


class Batch(ctypes.Structure):
    _fields_ = [
        ("nrep", ctypes.c_int32),
        ("tile_atoms", ctypes.c_int32),
        ("offsets", ctypes.c_void_p),
        ("boxes", ctypes.c_void_p),
        ("d_offsets", ctypes.c_void_p),
        ("d_boxes", ctypes.c_void_p),
    ]


class BatchTuning(ctypes.Structure):
    _fields_ = [
        ("lanes_per_atom", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("persistent", ctypes.c_int32),
        ("tile_atoms", ctypes.c_int32),
    ]


class LjmdError(RuntimeError):
    """A negative return code of a libljmd entry point."""

    def __init__(self, code, what, detail=""):
        self.code = code
        msg = f"{what}: {strerror(code)} ({code})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


_lib = None

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_u32 = ctypes.c_uint32
_sz = ctypes.c_size_t
_d = ctypes.c_double
_pbox = ctypes.POINTER(Box)
_pprm = ctypes.POINTER(Params)
_pnl = ctypes.POINTER(NList)
_pbat = ctypes.POINTER(Batch)
_ptun = ctypes.POINTER(BatchTuning)

SIGNATURES = {
    "ljmd_nlist_entries": (_i64, [_i64, _i32]),
    "ljmd_workspace_bytes": (_sz, [_i64, _pbox, _pprm, _u32]),
    "ljmd_nlist_aux_bytes": (_sz, [_i64, _pbox, _pprm]),
    "ljmd_nl_export": (ctypes.c_int, [_pnl, _vp, _vp, _vp]),
    "ljmd_nl_export_indices": (ctypes.c_int, [_pnl, _vp, _vp, _vp]),
    "ljmd_nl_build": (ctypes.c_int, [_vp, _vp, _i64, _pbox, _pprm, _pnl, _vp, _sz, _vp]),
    "ljmd_lj_forces": (ctypes.c_int, [_vp, _vp, _i64, _pbox, _pprm, _pnl, _u32, _vp, _vp, _vp,
                                      _sz, _vp]),
    "ljmd_lj_backward": (ctypes.c_int, [_vp, _vp, _i64, _pbox, _pprm, _pnl, _vp, _u32, _vp, _vp,
                                        _vp, _vp, _sz, _vp]),
    "ljmd_fm_grad": (ctypes.c_int, [_vp, _vp, _i64, _pbox, _pprm, _pnl, _vp, _vp, _u32, _vp, _vp,
                                    _vp, _vp, _vp, _sz, _vp]),
    "ljmd_batch_fm_grad": (ctypes.c_int, [_vp, _vp, _pbat, _pprm, _pnl, _vp, _vp, _u32, _vp, _vp,
                                          _vp, _vp, _vp, _sz, _vp]),
    "ljmd_lj_backward_noalloc": (ctypes.c_int, [_vp, _vp, _i64, _pbox, _pprm, _pnl, _vp, _u32,
                                                _vp, _vp, _vp, _vp]),
    "ljmd_md_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _i64, _pbox, _pprm, _pnl, _d, _i64,
                                    _i64, _i32, _i32, _u32, _vp, _vp, _sz, _vp]),
    "ljmd_batch_workspace_bytes": (_sz, [_pbat, _pprm, _u32]),
    "ljmd_batch_aux_bytes": (_sz, [_pbat, _pprm]),
    "ljmd_batch_nl_build": (ctypes.c_int, [_vp, _vp, _pbat, _pprm, _pnl, _vp, _sz, _vp]),
    "ljmd_batch_nl_export": (ctypes.c_int, [_pnl, _pbat, _pprm, _vp, _vp, _vp, _sz, _vp]),
    "ljmd_batch_lj_forces": (ctypes.c_int, [_vp, _vp, _pbat, _pprm, _pnl, _u32, _vp, _vp, _vp,
                                            _sz, _vp]),
    "ljmd_batch_lj_backward": (ctypes.c_int, [_vp, _vp, _pbat, _pprm, _pnl, _vp, _u32, _vp, _vp,
                                              _vp, _vp, _sz, _vp]),
    "ljmd_batch_md_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _pbat, _pprm, _pnl, _d, _i64,
                                          _i64, _i32, _i32, _u32, _vp, _vp, _sz, _vp]),
    "ljmd_batch_autotune": (ctypes.c_int, [_vp, _vp, _pbat, _pprm, _pnl, _u32, _vp, _vp, _sz,
                                           _vp, _ptun]),
    "ljmd_batch_set_tuning": (ctypes.c_int, [_pbat, _pprm, _u32, _ptun]),
    "ljmd_set_gather_lanes": (ctypes.c_int, [ctypes.c_int]),
    "ljmd_get_gather_lanes": (ctypes.c_int, []),
    "ljmd_nl_gather_lanes": (ctypes.c_int, [_pnl, _pbox, _pprm]),
    "ljmd_get_status": (ctypes.c_int, [_pnl, ctypes.POINTER(ctypes.c_int32), _vp]),
    "ljmd_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "ljmd_last_hip_error": (ctypes.c_char_p, []),
    "ljmd_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "ljmd_profile_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64)]),
}

PHASES = ("force", "build", "integrate", "other")


def header_functions():
    """Names of the functions declared in include/ljmd.h."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ljmd_[a-z_]+)\s*\(", text)))


def load():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"libljmd.so not found at {LIB_PATH}; build it with "
                "`python -m paper_2508_13523_amd.build` (or __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def strerror(code):
    return load().ljmd_strerror(int(code)).decode()


def last_hip_error():
    return load().ljmd_last_hip_error().decode()


def check(code, what):
    if code != OK:
        raise LjmdError(code, what, last_hip_error() if code == EHIP else "")
    return code


def check_value(code, what):
    """A non-negative result passes through; a negative one raises."""
    if code < 0:
        raise LjmdError(code, what, last_hip_error() if code == EHIP else "")
    return code
