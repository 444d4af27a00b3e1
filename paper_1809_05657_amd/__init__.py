"""Python binding of libhdarray.so, the MI355X HDArray runtime.

Argument marshalling only: every step of the ApplyKernel path (communication
set, pack, unpack, kernel, GDEF update) runs in the library's HIP kernels.
PyTorch is used, when present, only as the device-memory allocator and to
hand over the current stream.  The library must be built (``build.py``); a
missing library raises ImportError — there is no fallback.

Method names follow the paper's Table 2 (create, partition, apply = ApplyKernel,
read, write, reduce, set_absolute = SetAbsoluteUse/Def, set_trapezoid =
SetTrapezoidUse/Def) with the conventions of include/hdarray.h.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhdarray.so")

HOST = 63
STAR = -(2 ** 31)
F32, I32, F64 = 0, 1, 2
ROW, COL, BLOCK = 0, 1, 2
SUM, PROD, MAX, MIN = 0, 1, 2, 3
K_JACOBI2D, K_COPY, K_MATMUL, K_TRI2D, K_STENCIL3D7, K_CONV2D9 = 1, 2, 3, 4, 5, 6
BUILTIN_NAMES = {K_JACOBI2D: "jacobi2d", K_COPY: "copy", K_MATMUL: "matmul", K_TRI2D: "tri2d",
                 K_STENCIL3D7: "stencil3d7", K_CONV2D9: "conv2d9"}
EINVAL, EBOUNDS, ERACE, EKERNEL, ENOMEM, EHIP, ESTATE, ECAPACITY, ENOPLAN = -1, -2, -3, -4, -5, -6, -7, -8, -9
MSG_FIELDS = ("arg", "array", "src", "dst", "lo0", "lo1", "lo2", "hi0", "hi1", "hi2", "off", "bytes")
_TYPE_NAME = {F32: b"float", I32: b"int", F64: b"double"}
_DT = {F32: np.float32, I32: np.int32, F64: np.float64}


class HDArrayError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what} failed: {code}")
        self.code = code


class _Arg(C.Structure):
    class _V(C.Union):
        _fields_ = [("array", C.c_void_p), ("f", C.c_double), ("i", C.c_int64)]

    _fields_ = [("kind", C.c_int32), ("pad", C.c_int32), ("v", _V)]


class Stats(C.Structure):
    _fields_ = [("calls", C.c_int64), ("last_messages", C.c_int64), ("last_bytes", C.c_int64),
                ("total_messages", C.c_int64), ("total_bytes", C.c_int64), ("plans_built", C.c_int64),
                ("stencil_rows", C.c_int64), ("stencil_waves", C.c_int64),
                ("cache_hits", C.c_int64), ("cache_misses", C.c_int64), ("stencil_order", C.c_int64),
                ("allocs", C.c_int64), ("stencil_vec", C.c_int64), ("cache_gdef_hits", C.c_int64)]


class Profile(C.Structure):
    _fields_ = [("ms", C.c_double * 5), ("count", C.c_int64 * 5)]


PHASES = ("derive+gdef", "pack", "unpack", "kernel", "adjoint")
_lib = None
_TORCH_CB = None
_ALLOC_T = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_T = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


def exported_symbols():
    """Names declared in include/hdarray.h (for the export check)."""
    import re
    hdr = os.path.join(HERE, "..", "include", "hdarray.h")
    txt = open(hdr).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hdarray_[a-z_0-9]+)\s*\(", txt)))


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1809_05657_amd/build.py")
    L = C.CDLL(LIB_PATH)
    P, I64P = C.c_void_p, C.POINTER(C.c_int64)
    sig = {
        "hdarray_init": (C.c_int, [C.c_int, C.c_void_p, C.c_char_p, C.c_char_p]),
        "hdarray_exit": (None, []),
        "hdarray_show_device_info": (None, [C.c_int]),
        "hdarray_create": (P, [C.c_char_p, C.c_char_p, P, C.c_int, I64P]),
        "hdarray_array_id": (C.c_int, [P]),
        "hdarray_partition": (C.c_int, [C.c_int, C.c_int, I64P, I64P, I64P, C.c_int]),
        "hdarray_partition_manual": (C.c_int, [C.c_int, C.c_int, I64P, I64P]),
        "hdarray_partition_region": (C.c_int, [C.c_int, C.c_int, I64P, I64P]),
        "hdarray_register_kernel": (C.c_int, [C.c_char_p, C.c_char_p]),
        "hdarray_set_offsets": (C.c_int, [C.c_char_p, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int32)]),
        "hdarray_set_absolute_use": (C.c_int, [C.c_char_p, C.c_int, P, C.c_int, C.c_int, I64P, I64P]),
        "hdarray_set_absolute_def": (C.c_int, [C.c_char_p, C.c_int, P, C.c_int, C.c_int, I64P, I64P]),
        "hdarray_set_trapezoid_use": (C.c_int, [C.c_char_p, C.c_int, P, C.c_int, I64P]),
        "hdarray_set_trapezoid_def": (C.c_int, [C.c_char_p, C.c_int, P, C.c_int, I64P]),
        "hdarray_clear_sections": (C.c_int, [C.c_char_p, C.c_int, P, C.c_int]),
        "hdarray_apply_kernel": (C.c_int, [C.c_char_p, C.c_int, C.c_int, C.POINTER(_Arg)]),
        "hdarray_write": (C.c_int, [P, P, C.c_int]),
        "hdarray_read": (C.c_int, [P, P, C.c_int]),
        "hdarray_reduce": (C.c_int, [P, P, C.c_int, C.c_int]),
        "hdarray_reduce_noalloc": (C.c_int, [P, P, C.c_int, C.c_int]),
        "hdarray_set_stream": (C.c_int, [P]),
        "hdarray_set_allocator": (C.c_int, [_ALLOC_T, _FREE_T, P]),
        "hdarray_sync": (C.c_int, []),
        "hdarray_last_error": (C.c_int, []),
        "hdarray_error_string": (C.c_char_p, [C.c_int]),
        "hdarray_get_stats": (C.c_int, [C.POINTER(Stats)]),
        "hdarray_debug_messages": (C.c_int64, [I64P, C.c_int64]),
        "hdarray_debug_pack": (C.c_int64, [P, C.c_int64]),
        "hdarray_debug_gdef": (C.c_int, [P, P, P]),
        "hdarray_debug_device_buffer": (C.c_int, [P, C.c_int, P]),
        "hdarray_device_ptr": (P, [P, C.c_int]),
        "hdarray_profile": (C.c_int, [C.c_int]),
        "hdarray_set_plan_cache": (C.c_int, [C.c_int]),
        "hdarray_set_stencil_shape": (C.c_int, [C.c_int, C.c_int, C.c_int]),
        "hdarray_apply_adjoint": (C.c_int, [C.c_char_p, C.c_int, P, P, P, C.POINTER(C.c_float), P]),
        "hdarray_write_device": (C.c_int, [P, P, C.c_int]),
        "hdarray_read_device": (C.c_int, [P, P, C.c_int]),
        "hdarray_batch_begin": (C.c_int, []),
        "hdarray_batch_end": (C.c_int, []),
        "hdarray_batch_run": (C.c_int, [C.c_int]),
        "hdarray_batch_autotune": (C.c_int, [C.POINTER(C.c_int), C.c_int, C.c_int]),
        "hdarray_batch_phase_us": (C.c_int, [C.c_int, C.POINTER(C.c_double), C.c_int]),
        "hdarray_profile_read": (C.c_int, [C.POINTER(Profile)]),
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


class Array:
    def __init__(self, rt, handle, type_, shape):
        self.rt, self.h, self.type, self.shape = rt, handle, type_, tuple(shape)
        self.dtype = _DT[type_]
        self.id = rt.L.hdarray_array_id(handle)
        self.N = int(np.prod(shape))


class Runtime:
    """The process-wide runtime (one per process; creating a new one calls
    HDArrayExit on the previous state)."""

    def __init__(self, use_torch_allocator=True, row_cap=None, stream=None, windows=None):
        self.L = load()
        self.L.hdarray_exit()
        if use_torch_allocator:
            self._install_torch_allocator()
        argv = []
        if row_cap:
            argv.append(f"--hd-row-cap={int(row_cap)}".encode())
        if windows is not None:
            if windows not in ("full", "compact"):
                raise ValueError("windows must be 'full' or 'compact'")
            argv.append(f"--hd-windows={windows}".encode())
        arr = (C.c_char_p * max(len(argv), 1))(*argv)
        self._ck(self.L.hdarray_init(len(argv), C.cast(arr, C.c_void_p), None, None), "init")
        if stream is not None:
            self.L.hdarray_set_stream(C.c_void_p(stream))
        self.kernels = {}
        self.arrays = []

    def _install_torch_allocator(self):
        global _TORCH_CB
        try:
            import torch
        except ImportError:  # plain hipMalloc
            return
        if not torch.cuda.is_available():
            return
        if _TORCH_CB is None:
            dev = torch.cuda.current_device()

            def _alloc(n, ctx):
                return torch.cuda.caching_allocator_alloc(int(n), dev, 0)

            def _free(p, ctx):
                torch.cuda.caching_allocator_delete(p)

            # module-level: the library keeps calling them across runtimes
            _TORCH_CB = (_ALLOC_T(_alloc), _FREE_T(_free))
        self.L.hdarray_set_allocator(_TORCH_CB[0], _TORCH_CB[1], None)

    def _ck(self, rc, what):
        if rc < 0:
            raise HDArrayError(rc, what)
        return rc

    def close(self):
        self.L.hdarray_exit()

    # -- Table 2 ------------------------------------------------------------
    def create(self, data=None, shape=None, type_=F32, name="a"):
        if data is not None:
            data = np.ascontiguousarray(data, dtype=_DT[type_])
            shape = data.shape
        sz, szp = _i64(shape)
        h = self.L.hdarray_create(name.encode(), _TYPE_NAME[type_], data.ctypes.data if data is not None else None,
                                  len(shape), szp)
        if not h:
            raise HDArrayError(self.L.hdarray_last_error(), "create")
        a = Array(self, h, type_, shape)
        self.arrays.append(a)
        return a

    def partition(self, kind, sizes, lo=None, hi=None, ndev=1):
        dim = len(sizes)
        lo = [0] * dim if lo is None else lo
        hi = list(sizes) if hi is None else hi
        s, sp = _i64(sizes)
        l, lp = _i64(lo)
        h, hp = _i64(hi)
        return self._ck(self.L.hdarray_partition(kind, dim, sp, lp, hp, ndev), "partition")

    def partition_manual(self, los, his):
        los = np.asarray(los, dtype=np.int64)
        his = np.asarray(his, dtype=np.int64)
        ndev, dim = los.shape
        l, lp = _i64(los.ravel())
        h, hp = _i64(his.ravel())
        return self._ck(self.L.hdarray_partition_manual(dim, ndev, lp, hp), "partition_manual")

    def part_region(self, part, dev):
        lo, lp = _i64([0, 0, 0])
        hi, hp = _i64([0, 0, 0])
        self._ck(self.L.hdarray_partition_region(part, dev, lp, hp), "part_region")
        return tuple(int(x) for x in lo), tuple(int(x) for x in hi)

    def kernel(self, name, builtin):
        b = BUILTIN_NAMES[builtin] if isinstance(builtin, int) else builtin
        k = self._ck(self.L.hdarray_register_kernel(name.encode(), b.encode()), "register_kernel")
        self.kernels[name] = k
        return k

    def set_offsets(self, kname, arg, use_or_def, offsets):
        raw = np.zeros((max(len(offsets), 1), 3), dtype=np.int32)
        for i, o in enumerate(offsets):
            for j, v in enumerate(o):
                raw[i, j] = STAR if (v is None or v == "*") else int(v)
        self._ck(self.L.hdarray_set_offsets(kname.encode(), arg, use_or_def, len(offsets),
                                            raw.ctypes.data_as(C.POINTER(C.c_int32))), "set_offsets")

    def set_absolute(self, kname, part, arr, dev, use_or_def, lo, hi):
        l, lp = _i64(lo)
        h, hp = _i64(hi)
        f = self.L.hdarray_set_absolute_def if use_or_def else self.L.hdarray_set_absolute_use
        self._ck(f(kname.encode(), part, arr.h, dev, len(lo), lp, hp), "set_absolute")

    def set_trapezoid(self, kname, part, arr, dev, use_or_def, corners):
        cc, cp = _i64(np.asarray(corners).ravel())
        f = self.L.hdarray_set_trapezoid_def if use_or_def else self.L.hdarray_set_trapezoid_use
        self._ck(f(kname.encode(), part, arr.h, dev, cp), "set_trapezoid")

    def clear_sections(self, kname, part, arr, dev=-1):
        self._ck(self.L.hdarray_clear_sections(kname.encode(), part, arr.h, dev), "clear_sections")

    def apply(self, kname, part, arrs, scalars=()):
        n = len(arrs) + len(scalars)
        args = (_Arg * n)()
        for i, a in enumerate(arrs):
            args[i].kind = 0
            args[i].v.array = a.h
        for j, s in enumerate(scalars):
            args[len(arrs) + j].kind = 1
            args[len(arrs) + j].v.f = float(s)
        return self._ck(self.L.hdarray_apply_kernel(kname.encode(), part, n, args), "apply_kernel")

    def write(self, arr, data, part):
        data = np.ascontiguousarray(data, dtype=arr.dtype).reshape(arr.shape)
        self._ck(self.L.hdarray_write(arr.h, data.ctypes.data, part), "write")

    def read(self, arr, part, out=None):
        out = np.zeros(arr.shape, dtype=arr.dtype) if out is None else out
        self._ck(self.L.hdarray_read(arr.h, out.ctypes.data, part), "read")
        return out

    def reduce(self, arr, op, part):
        res = np.zeros(1, dtype=arr.dtype)
        self._ck(self.L.hdarray_reduce(arr.h, res.ctypes.data, op, part), "reduce")
        return res[0].item()

    def reduce_noalloc(self, arr, op, part):
        """hdarray_reduce_noalloc: as reduce, with no allocation (the plan of
        (arr, part) must come from an earlier reduce)."""
        res = np.zeros(1, dtype=arr.dtype)
        self._ck(self.L.hdarray_reduce_noalloc(arr.h, res.ctypes.data, op, part), "reduce_noalloc")
        return res[0].item()

    def sync(self):
        return self._ck(self.L.hdarray_sync(), "sync")

    def stats(self):
        st = Stats()
        self._ck(self.L.hdarray_get_stats(C.byref(st)), "get_stats")
        return {f: getattr(st, f) for f, _ in Stats._fields_}

    def apply_adjoint(self, kname, part, du_in, du_out, u, coeffs, cbar_ptr=None):
        cf = (C.c_float * 7)(*[float(c) for c in coeffs])
        return self._ck(self.L.hdarray_apply_adjoint(kname.encode(), part, du_in.h, du_out.h, u.h, cf,
                                                     C.c_void_p(cbar_ptr) if cbar_ptr else None), "apply_adjoint")

    def write_device(self, arr, dptr, part):
        self._ck(self.L.hdarray_write_device(arr.h, C.c_void_p(dptr), part), "write_device")

    def read_device(self, arr, dptr, part):
        self._ck(self.L.hdarray_read_device(arr.h, C.c_void_p(dptr), part), "read_device")

    def batch_begin(self):
        self._ck(self.L.hdarray_batch_begin(), "batch_begin")

    def batch_end(self):
        return self._ck(self.L.hdarray_batch_end(), "batch_end")

    def batch_run(self, bid):
        self._ck(self.L.hdarray_batch_run(bid), "batch_run")

    def batch_phase_us(self, batch):
        buf = (C.c_double * 16)()
        n = self._ck(self.L.hdarray_batch_phase_us(batch, buf, 16), "batch_phase_us")
        return [buf[i] for i in range(n)]

    def batch_autotune(self, ids, reps=2):
        arr = (C.c_int * len(ids))(*ids)
        return self._ck(self.L.hdarray_batch_autotune(arr, len(ids), reps), "batch_autotune")

    def set_stencil_shape(self, rows=0, waves=0, order=1):
        """Fix the 2-D stencil tile shape (rows 4/8/16 with waves 1/4 and
        tile order 1 along rows / 0 down columns, or strips of 32/64 rows);
        (0, 0) restores timing-based selection."""
        self._ck(self.L.hdarray_set_stencil_shape(int(rows), int(waves), int(order)), "set_stencil_shape")

    def set_plan_cache(self, on=True):
        """Reuse a plan's message table while its arrays' GDEF is unchanged
        (Sec. 4.2); off by default."""
        self._ck(self.L.hdarray_set_plan_cache(int(bool(on))), "set_plan_cache")

    def profile(self, enable=True):
        self._ck(self.L.hdarray_profile(int(enable)), "profile")

    def profile_read(self):
        pr = Profile()
        self._ck(self.L.hdarray_profile_read(C.byref(pr)), "profile_read")
        return {PHASES[i]: (pr.ms[i], pr.count[i]) for i in range(len(PHASES))}

    # -- parity dumps ------------------------------------------------------------
    def messages(self):
        n = self._ck(self.L.hdarray_debug_messages(None, 0), "debug_messages")
        out = np.zeros((max(n, 1), len(MSG_FIELDS)), dtype=np.int64)
        self._ck(self.L.hdarray_debug_messages(out.ctypes.data_as(C.POINTER(C.c_int64)), n), "debug_messages")
        return out[:n]

    def pack(self):
        n = self._ck(self.L.hdarray_debug_pack(None, 0), "debug_pack")
        out = np.zeros(max(n, 1), dtype=np.uint8)
        self._ck(self.L.hdarray_debug_pack(out.ctypes.data, n), "debug_pack")
        return out[:n]

    def gdef(self, arr):
        owner = np.zeros(arr.N, dtype=np.int8)
        holders = np.zeros(arr.N, dtype=np.uint64)
        self._ck(self.L.hdarray_debug_gdef(arr.h, owner.ctypes.data, holders.ctypes.data), "debug_gdef")
        return owner.reshape(arr.shape), holders.reshape(arr.shape)

    def device_buffer(self, arr, dev):
        out = np.zeros(arr.shape, dtype=arr.dtype)
        self._ck(self.L.hdarray_debug_device_buffer(arr.h, dev, out.ctypes.data), "debug_device_buffer")
        return out

    def device_ptr(self, arr, dev):
        p = self.L.hdarray_device_ptr(arr.h, dev)
        if not p:
            raise HDArrayError(self.L.hdarray_last_error(), "device_ptr")
        return p
