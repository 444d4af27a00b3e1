"""CPU oracle for the HDArray ApplyKernel path — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it,
and it shares no code with the HIP path: the C core (``hdoracle.c``) is a
plain, per-element, brute-force implementation of the paper's definitions
(arXiv 1809.05657, Sec. 2.1-2.2, Eq. 1-4, Sec. 3.1 Table 2).

Conventions (same reading as the product, written independently):
  * endpoints 0..62 are logical devices, 63 is the host;
  * rectangles are half-open in normalised (planes, rows, cols) coordinates;
  * messages are ordered by array argument, then row-major lower corner,
    then destination; pack offsets are in bytes, aligned to the element size.

Every function is pinned by a CPU test against the paper or the mathematics
(tests/test_oracle_pins.py, tests/test_oracle_pins_exact.py): hand-derived
message lists and trapezoid rows, Table 3 volumes, closed forms, an exact
rational evaluation of the FP32 operation chains, exact products for the
reductions.  A function without such a pin would be marked "parity
unpinned" in its docstring; none is.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

HOST = 63
STAR = -(2 ** 31)
F32, I32, F64 = 0, 1, 2
ROW, COL, BLOCK = 0, 1, 2
SUM, PROD, MAX, MIN = 0, 1, 2, 3
K_JACOBI2D, K_COPY, K_MATMUL, K_TRI2D, K_STENCIL3D7, K_CONV2D9 = 1, 2, 3, 4, 5, 6
EINVAL, EBOUNDS, ERACE, EKERNEL, ENOMEM, ESTATE, ECOHERENCE = -1, -2, -3, -4, -5, -7, -9
MSG_FIELDS = ("arg", "array", "src", "dst", "lo0", "lo1", "lo2", "hi0", "hi1", "hi2", "off", "bytes")

_DT = {F32: np.float32, I32: np.int32, F64: np.float64}
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB) or os.path.getmtime(_build.LIB) < os.path.getmtime(
            os.path.join(os.path.dirname(_build.LIB), "hdoracle.c")):
        _build.build()
    L = C.CDLL(_build.LIB)
    P, I64P = C.c_void_p, C.POINTER(C.c_int64)
    sig = {
        "orc_new": (P, []), "orc_free": (None, [P]), "orc_set_mode": (None, [P, C.c_int, C.c_int]),
        "orc_create": (C.c_int, [P, C.c_int, C.c_int, I64P, P]),
        "orc_partition": (C.c_int, [P, C.c_int, C.c_int, I64P, I64P, I64P, C.c_int]),
        "orc_partition_manual": (C.c_int, [P, C.c_int, C.c_int, I64P, I64P]),
        "orc_part_region": (C.c_int, [P, C.c_int, C.c_int, I64P, I64P]),
        "orc_kernel": (C.c_int, [P, C.c_char_p, C.c_int]),
        "orc_set_offsets": (C.c_int, [P, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int32)]),
        "orc_set_absolute": (C.c_int, [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, I64P, I64P]),
        "orc_set_trapezoid": (C.c_int, [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, I64P]),
        "orc_clear_sections": (C.c_int, [P, C.c_int, C.c_int, C.c_int, C.c_int]),
        "orc_apply": (C.c_int, [P, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), C.c_int,
                                C.POINTER(C.c_double)]),
        "orc_write": (C.c_int, [P, C.c_int, P, C.c_int]),
        "orc_read": (C.c_int, [P, C.c_int, P, C.c_int]),
        "orc_reduce": (C.c_int, [P, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double), I64P]),
        "orc_last_nmsgs": (C.c_int64, [P]),
        "orc_last_messages": (C.c_int64, [P, I64P, C.c_int64]),
        "orc_last_pack_bytes": (C.c_int64, [P]),
        "orc_last_pack": (C.c_int64, [P, P, C.c_int64]),
        "orc_gdef": (C.c_int, [P, C.c_int, P, P]),
        "orc_truth": (C.c_int, [P, C.c_int, P]),
        "orc_truth64": (C.c_int, [P, C.c_int, P]),
        "orc_device_buffer": (C.c_int, [P, C.c_int, C.c_int, P]),
        "orc_bad_reads": (C.c_int64, [P]),
        "orc_inject_drop": (None, [P, C.c_int64]),
        "orc_s3d_forward64": (None, [I64P, P, P, C.c_int, P]),
        "orc_threads": (C.c_int, []),
        "orc_s3d_adjoint64": (None, [I64P, P, P, C.c_int, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _i64(v):
    a = np.ascontiguousarray(np.asarray(v, dtype=np.int64))
    return a, a.ctypes.data_as(C.POINTER(C.c_int64))


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what} failed with code {code}")
        self.code = code


def _ck(rc, what):
    if rc < 0:
        raise OracleError(rc, what)
    return rc


class Array:
    def __init__(self, orc, aid, type_, shape):
        self.orc, self.id, self.type, self.shape = orc, aid, type_, tuple(shape)
        self.dtype = _DT[type_]
        n = list(shape)
        self.nshape = tuple([1] * (3 - len(n)) + n)
        self.N = int(np.prod(shape))


class Oracle:
    """One oracle run (one HDArray program).  Methods follow Table 2."""

    def __init__(self, simulate_devices=True, eval_kernels=True):
        self.L = _load()
        self.c = self.L.orc_new()
        self.L.orc_set_mode(self.c, int(simulate_devices), int(eval_kernels))
        self.kernels = {}
        self.arrays = []

    def close(self):
        if self.c:
            self.L.orc_free(self.c)
            self.c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- Table 2 ------------------------------------------------------------
    def create(self, data=None, shape=None, type_=F32):
        if data is not None:
            data = np.ascontiguousarray(data, dtype=_DT[type_])
            shape = data.shape
        sz, szp = _i64(shape)
        ptr = data.ctypes.data if data is not None else None
        aid = _ck(self.L.orc_create(self.c, type_, len(shape), szp, ptr), "create")
        a = Array(self, aid, type_, shape)
        a._keep = data
        self.arrays.append(a)
        return a

    def partition(self, kind, sizes, lo=None, hi=None, ndev=1):
        dim = len(sizes)
        lo = [0] * dim if lo is None else lo
        hi = list(sizes) if hi is None else hi
        s, sp = _i64(sizes)
        l, lp = _i64(lo)
        h, hp = _i64(hi)
        return _ck(self.L.orc_partition(self.c, kind, dim, sp, lp, hp, ndev), "partition")

    def partition_manual(self, los, his):
        los = np.asarray(los, dtype=np.int64)
        his = np.asarray(his, dtype=np.int64)
        ndev, dim = los.shape
        l, lp = _i64(los.ravel())
        h, hp = _i64(his.ravel())
        return _ck(self.L.orc_partition_manual(self.c, dim, ndev, lp, hp), "partition_manual")

    def part_region(self, part, dev):
        lo, lp = _i64([0, 0, 0])
        hi, hp = _i64([0, 0, 0])
        _ck(self.L.orc_part_region(self.c, part, dev, lp, hp), "part_region")
        return tuple(lo), tuple(hi)

    def kernel(self, name, builtin):
        k = _ck(self.L.orc_kernel(self.c, name.encode(), builtin), "kernel")
        self.kernels[name] = k
        return k

    def set_offsets(self, kname, arg, use_or_def, offsets):
        """offsets: list of per-dimension tuples; None or '*' = whole dimension"""
        raw = np.zeros((max(len(offsets), 1), 3), dtype=np.int32)
        for i, o in enumerate(offsets):
            for j, v in enumerate(o):
                raw[i, j] = STAR if (v is None or v == "*") else int(v)
        p = raw.ctypes.data_as(C.POINTER(C.c_int32))
        _ck(self.L.orc_set_offsets(self.c, self.kernels[kname], arg, use_or_def, len(offsets), p),
            "set_offsets")

    def set_absolute(self, kname, part, arr, dev, use_or_def, lo, hi):
        l, lp = _i64(lo)
        h, hp = _i64(hi)
        _ck(self.L.orc_set_absolute(self.c, self.kernels[kname], part, arr.id, dev, use_or_def, lp, hp),
            "set_absolute")

    def set_trapezoid(self, kname, part, arr, dev, use_or_def, corners):
        cc, cp = _i64(np.asarray(corners).ravel())
        _ck(self.L.orc_set_trapezoid(self.c, self.kernels[kname], part, arr.id, dev, use_or_def, cp),
            "set_trapezoid")

    def clear_sections(self, kname, part, arr, dev=-1):
        _ck(self.L.orc_clear_sections(self.c, self.kernels[kname], part, arr.id, dev), "clear_sections")

    def apply(self, kname, part, arrs, scalars=()):
        ids = (C.c_int * len(arrs))(*[a.id for a in arrs])
        sc = (C.c_double * max(len(scalars), 1))(*scalars)
        return _ck(self.L.orc_apply(self.c, self.kernels[kname], part, len(arrs), ids, len(scalars), sc),
                   "apply")

    def write(self, arr, data, part):
        data = np.ascontiguousarray(data, dtype=arr.dtype).reshape(arr.shape)
        _ck(self.L.orc_write(self.c, arr.id, data.ctypes.data, part), "write")

    def read(self, arr, part, out=None):
        out = np.zeros(arr.shape, dtype=arr.dtype) if out is None else out
        _ck(self.L.orc_read(self.c, arr.id, out.ctypes.data, part), "read")
        return out

    def reduce(self, arr, op, part):
        rf = C.c_double(0.0)
        ri = C.c_int64(0)
        _ck(self.L.orc_reduce(self.c, arr.id, op, part, C.byref(rf), C.byref(ri)), "reduce")
        return ri.value if arr.type == I32 else rf.value

    # -- dumps ----------------------------------------------------------------
    def messages(self):
        n = self.L.orc_last_nmsgs(self.c)
        out = np.zeros((max(n, 1), len(MSG_FIELDS)), dtype=np.int64)
        self.L.orc_last_messages(self.c, out.ctypes.data_as(C.POINTER(C.c_int64)), n)
        return out[:n]

    def pack(self):
        n = self.L.orc_last_pack_bytes(self.c)
        out = np.zeros(max(n, 1), dtype=np.uint8)
        self.L.orc_last_pack(self.c, out.ctypes.data, n)
        return out[:n]

    def gdef(self, arr):
        owner = np.zeros(arr.N, dtype=np.int8)
        holders = np.zeros(arr.N, dtype=np.uint64)
        _ck(self.L.orc_gdef(self.c, arr.id, owner.ctypes.data, holders.ctypes.data), "gdef")
        return owner.reshape(arr.shape), holders.reshape(arr.shape)

    def truth(self, arr):
        out = np.zeros(arr.shape, dtype=arr.dtype)
        _ck(self.L.orc_truth(self.c, arr.id, out.ctypes.data), "truth")
        return out

    def truth64(self, arr):
        out = np.zeros(arr.shape, dtype=np.float64)
        _ck(self.L.orc_truth64(self.c, arr.id, out.ctypes.data), "truth64")
        return out

    def device_buffer(self, arr, dev):
        out = np.zeros(arr.shape, dtype=arr.dtype)
        _ck(self.L.orc_device_buffer(self.c, arr.id, dev, out.ctypes.data), "device_buffer")
        return out

    def bad_reads(self):
        return self.L.orc_bad_reads(self.c)

    def inject_drop(self, idx):
        self.L.orc_inject_drop(self.c, idx)


def s3d_forward64(u0, coeffs, T):
    """FP64 whole-array forward of T 7-point stencil steps (fixed boundary)."""
    L = _load()
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    cf = np.ascontiguousarray(coeffs, dtype=np.float64)
    n, npp = _i64(u0.shape)
    out = np.zeros_like(u0)
    L.orc_s3d_forward64(npp, u0.ctypes.data, cf.ctypes.data, T, out.ctypes.data)
    return out


def s3d_adjoint64(u0, coeffs, T, w):
    """FP64 reverse mode of L = sum(w * u_T): returns (dL/du0, dL/dc)."""
    L = _load()
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    cf = np.ascontiguousarray(coeffs, dtype=np.float64)
    n, npp = _i64(u0.shape)
    g = np.zeros_like(u0)
    gc = np.zeros(7)
    L.orc_s3d_adjoint64(npp, u0.ctypes.data, cf.ctypes.data, T, w.ctypes.data, g.ctypes.data,
                        gc.ctypes.data)
    return g, gc


def messages_as_dicts(msgs):
    return [dict(zip(MSG_FIELDS, map(int, m))) for m in msgs]


def threads():
    """OpenMP threads the oracle's loops use."""
    return int(_load().orc_threads())
