"""ctypes binding of include/sbqa.h (argument marshalling only).

Every function here has the name of the C entry point it wraps and does no
arithmetic of its own: all SBQA work runs in libsbqa.so on the GPU. The
library must have been built (``paper_2604_01050_amd.build``); importing this
module without it raises, there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsbqa.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EBUDGET, EAGAIN = 0, -1, -2, -3, -4, -5, -6
F_TERNARY, F_SIGN, F_BALLISTIC = 0, 1, 2
PREC_AUTO, PREC_FP32, PREC_FP8, PREC_BF16X3, PREC_INT8, PREC_FP4 = 0, 1, 2, 3, 4, 5
JP_LINEAR, JP_PAPER, JP_TABLE = 0, 1, 2
LOOP_AUTO, LOOP_STREAM, LOOP_RESIDENT = 0, 1, 2
JPACK_AUTO, JPACK_BYTES = 0, 1
REORDER_AUTO, REORDER_OFF, REORDER_ON = 0, 1, 2
PATHS = {0: "dense_fp32", 1: "dense_fp8", 2: "dense_bf16x3", 3: "csr_fp32", 4: "dense_int8", 5: "dense_fp8_packed",
         6: "dense_fp4", 7: "dense_fp4_packed"}
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE", -5: "EBUDGET", -6: "EAGAIN"}


class SbqaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_STATUS.get(status, status), message))
        self.status = status
        self.message = message


class Coupling(ct.Structure):
    _fields_ = [("dense", ct.c_void_p), ("row_ptr", ct.c_void_p), ("col", ct.c_void_p),
                ("val", ct.c_void_p), ("nnz", ct.c_int64), ("n3", ct.c_int64), ("tri", ct.c_void_p),
                ("K", ct.c_void_p)]


class Schedule(ct.Structure):
    _fields_ = [("steps", ct.c_uint32), ("dt", ct.c_double), ("a0", ct.c_double), ("c0", ct.c_double),
                ("fmode", ct.c_int32), ("delta_max", ct.c_double), ("jp_kind", ct.c_int32),
                ("jp_start", ct.c_double), ("jp_end", ct.c_double), ("gamma0_over_R", ct.c_double),
                ("beta_lo", ct.c_double), ("beta_hi", ct.c_double), ("alpha_lo", ct.c_double),
                ("alpha_hi", ct.c_double), ("beta", ct.c_void_p), ("alpha", ct.c_void_p),
                ("jp_table", ct.c_void_p), ("seed", ct.c_uint64), ("init_amp", ct.c_double),
                ("precision", ct.c_int32), ("energy_every", ct.c_uint32), ("loop_kernel", ct.c_int32),
                ("dense_tile", ct.c_int32), ("j_packing", ct.c_int32), ("reorder", ct.c_int32)]


class Info(ct.Structure):
    _fields_ = [("N", ct.c_int32), ("R", ct.c_int32), ("runs", ct.c_int32), ("steps", ct.c_uint32),
                ("step", ct.c_uint32), ("path", ct.c_int32), ("fmode", ct.c_int32), ("c0", ct.c_double),
                ("j_integral", ct.c_int32), ("device_bytes", ct.c_size_t), ("resident", ct.c_int32),
                ("tile_cols", ct.c_int32), ("reordered", ct.c_int32)]


def _load() -> ct.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsbqa.so is not built (run paper_2604_01050_amd.build.build()); "
                          "there is no fallback path")
    # PyTorch ships its own HIP runtime: loaded first, it is the one the
    # library binds to, so the process holds one runtime (loading the library
    # first left two, and the library's could not use PyTorch's streams and
    # reported too few co-resident workgroups for the resident loop)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ct.CDLL(LIB_PATH)
    vp, i32, u32, u64, d = ct.c_void_p, ct.c_int32, ct.c_uint32, ct.c_uint64, ct.c_double
    sig = {
        "sbqa_schedule_default": ([], Schedule),
        "sbqa_create": ([ct.POINTER(Coupling), vp, i32, i32, i32, ct.POINTER(Schedule), ct.POINTER(vp)], i32),
        "sbqa_step": ([vp, u32], i32),
        "sbqa_best": ([vp, vp, vp], i32),
        "sbqa_best_step": ([vp, vp], i32),
        "sbqa_energy": ([vp, vp, i32, vp], i32),
        "sbqa_energy_noalloc": ([vp, vp, i32, vp], i32),
        "sbqa_fields": ([vp, vp], i32),
        "sbqa_get_state": ([vp, vp, vp], i32),
        "sbqa_set_state": ([vp, vp, vp], i32),
        "sbqa_run_params": ([vp, vp, vp], i32),
        "sbqa_jperp_table": ([vp, vp], i32),
        "sbqa_set_stream": ([vp, vp], i32),
        "sbqa_info": ([vp, ct.POINTER(Info)], i32),
        "sbqa_sync": ([vp], i32),
        "sbqa_inject_wait_timeout": ([vp], i32),
        "sbqa_last_error": ([], ct.c_char_p),
        "sbqa_destroy": ([vp], None),
        "sbqa_server_create": ([ct.c_size_t, i32, ct.POINTER(vp)], i32),
        "sbqa_submit": ([vp, ct.POINTER(Coupling), vp, i32, i32, i32, ct.POINTER(Schedule), ct.POINTER(u64)], i32),
        "sbqa_poll": ([vp, u64, vp, vp, vp], i32),
        "sbqa_server_stats": ([vp, vp, vp, vp], i32),
        "sbqa_server_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()


def sbqa_last_error() -> str:
    return lib.sbqa_last_error().decode()


def sbqa_schedule_default() -> Schedule:
    return lib.sbqa_schedule_default()


def _check(st: int) -> None:
    if st != OK:
        raise SbqaError(st, lib.sbqa_last_error().decode())


def _p(a):
    return None if a is None else a.ctypes.data


def make_schedule(**kw):
    """sbqa_schedule_default() with fields overridden; array fields (beta,
    alpha, jp_table) are returned as numpy arrays the caller keeps alive."""
    s = lib.sbqa_schedule_default()
    keep = []
    for k, v in kw.items():
        if k in ("beta", "alpha"):
            a = np.ascontiguousarray(v, dtype=np.float64)
            keep.append(a)
            setattr(s, k, a.ctypes.data)
        elif k == "jp_table":
            a = np.ascontiguousarray(v, dtype=np.float32)
            keep.append(a)
            s.jp_table = a.ctypes.data
        else:
            setattr(s, k, v)
    return s, keep


def _coupling(J=None, csr=None, tri=None, K=None):
    """tri (n3, 3) and K (n3,): optional three-body terms (CSR couplings)."""
    keep = []
    c = Coupling()
    if tri is not None:
        T = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
        Kd = np.ascontiguousarray(K, dtype=np.float64).reshape(-1)
        if Kd.size != T.shape[0]:
            raise ValueError("tri and K differ in length")
        keep += [T, Kd]
        c.n3, c.tri, c.K = Kd.size, T.ctypes.data, Kd.ctypes.data
    if J is not None:
        Jd = np.ascontiguousarray(J, dtype=np.float64)
        keep.append(Jd)
        c.dense = Jd.ctypes.data
        N = Jd.shape[0]
    else:
        rp = np.ascontiguousarray(csr[0], dtype=np.int32)
        col = np.ascontiguousarray(csr[1], dtype=np.int32)
        val = np.ascontiguousarray(csr[2], dtype=np.float64)
        keep += [rp, col, val]
        c.row_ptr, c.col, c.val, c.nnz = rp.ctypes.data, col.ctypes.data, val.ctypes.data, col.size
        N = rp.size - 1
    return c, keep, N


class Context:
    """Owns an sbqa_ctx*; shapes kept for output allocation."""

    def __init__(self, ptr, N, R, runs, steps):
        self.ptr, self.N, self.R, self.runs, self.steps = ptr, N, R, runs, steps
        self.C = R * runs

    def __del__(self):
        if getattr(self, "ptr", None):
            lib.sbqa_destroy(self.ptr)
            self.ptr = None


def sbqa_create(J=None, h=None, N=None, R=1, runs=1, schedule=None, csr=None, tri=None, K=None,
                **sched_kw) -> Context:
    if (J is None) == (csr is None):
        raise ValueError("give exactly one of J (dense) or csr=(row_ptr, col, val)")
    c, keep, n = _coupling(J, csr, tri, K)
    N = n if N is None else N
    if schedule is None:
        schedule, keep2 = make_schedule(**sched_kw)
        keep += keep2
    hd = None if h is None else np.ascontiguousarray(h, dtype=np.float64)
    out = ct.c_void_p()
    _check(lib.sbqa_create(ct.byref(c), _p(hd), N, R, runs, ct.byref(schedule), ct.byref(out)))
    return Context(out.value, N, R, runs, schedule.steps)


def sbqa_step(ctx: Context, n: int) -> None:
    _check(lib.sbqa_step(ctx.ptr, n))


def sbqa_best(ctx: Context):
    E = np.empty(ctx.runs, dtype=np.float64)
    s = np.empty((ctx.runs, ctx.N), dtype=np.int8)
    _check(lib.sbqa_best(ctx.ptr, _p(E), _p(s)))
    return E, s


def sbqa_best_step(ctx: Context):
    st = np.empty(ctx.runs, dtype=np.int64)
    _check(lib.sbqa_best_step(ctx.ptr, _p(st)))
    return st


def sbqa_energy(ctx: Context, spins) -> np.ndarray:
    s = np.ascontiguousarray(np.atleast_2d(spins), dtype=np.int8)
    E = np.empty(s.shape[0], dtype=np.float64)
    _check(lib.sbqa_energy(ctx.ptr, _p(s), s.shape[0], _p(E)))
    return E


def sbqa_energy_noalloc(ctx: Context, spins_ptr: int, count: int, out_ptr: int) -> None:
    """spins_ptr / out_ptr: device addresses (count*N int8, count float64);
    asynchronous on the context's stream."""
    _check(lib.sbqa_energy_noalloc(ctx.ptr, spins_ptr, count, out_ptr))


def sbqa_fields(ctx: Context) -> np.ndarray:
    phi = np.empty((ctx.N, ctx.C), dtype=np.float32)
    _check(lib.sbqa_fields(ctx.ptr, _p(phi)))
    return phi


def sbqa_get_state(ctx: Context):
    x = np.empty((ctx.N, ctx.C), dtype=np.float32)
    y = np.empty((ctx.N, ctx.C), dtype=np.float32)
    _check(lib.sbqa_get_state(ctx.ptr, _p(x), _p(y)))
    return x, y


def sbqa_set_state(ctx: Context, x, y) -> None:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    assert x.shape == (ctx.N, ctx.C) and y.shape == (ctx.N, ctx.C)
    _check(lib.sbqa_set_state(ctx.ptr, _p(x), _p(y)))


def sbqa_run_params(ctx: Context):
    b = np.empty(ctx.runs)
    a = np.empty(ctx.runs)
    _check(lib.sbqa_run_params(ctx.ptr, _p(b), _p(a)))
    return b, a


def sbqa_jperp_table(ctx: Context) -> np.ndarray:
    jp = np.empty((ctx.runs, ctx.steps), dtype=np.float32)
    _check(lib.sbqa_jperp_table(ctx.ptr, _p(jp)))
    return jp


def sbqa_set_stream(ctx: Context, stream) -> None:
    """stream: torch.cuda.Stream, a raw hipStream_t int, or None."""
    if stream is not None and not isinstance(stream, int):
        stream = stream.cuda_stream
    _check(lib.sbqa_set_stream(ctx.ptr, stream))


def sbqa_info(ctx: Context) -> dict:
    i = Info()
    _check(lib.sbqa_info(ctx.ptr, ct.byref(i)))
    return {"N": i.N, "R": i.R, "runs": i.runs, "steps": i.steps, "step": i.step,
            "path": PATHS[i.path], "fmode": i.fmode, "c0": i.c0, "j_integral": bool(i.j_integral),
            "device_bytes": i.device_bytes, "resident": bool(i.resident), "tile_cols": i.tile_cols,
            "reordered": bool(i.reordered)}


def sbqa_sync(ctx: Context) -> None:
    _check(lib.sbqa_sync(ctx.ptr))


def sbqa_inject_wait_timeout(ctx: Context) -> None:
    _check(lib.sbqa_inject_wait_timeout(ctx.ptr))


def sbqa_destroy(ctx: Context) -> None:
    if ctx.ptr:
        lib.sbqa_destroy(ctx.ptr)
        ctx.ptr = None


# ------------------------------------------------------------------ serving
class Server:
    def __init__(self, ptr):
        self.ptr = ptr
        self.shapes = {}

    def __del__(self):
        if getattr(self, "ptr", None):
            lib.sbqa_server_destroy(self.ptr)
            self.ptr = None


def sbqa_server_create(hbm_budget_bytes: int, max_slots: int) -> Server:
    out = ct.c_void_p()
    _check(lib.sbqa_server_create(int(hbm_budget_bytes), int(max_slots), ct.byref(out)))
    return Server(out.value)


def sbqa_submit(srv: Server, J=None, h=None, R=1, runs=1, schedule=None, csr=None, tri=None, K=None,
                **sched_kw) -> int:
    c, keep, N = _coupling(J, csr, tri, K)
    if schedule is None:
        schedule, keep2 = make_schedule(**sched_kw)
        keep += keep2
    hd = None if h is None else np.ascontiguousarray(h, dtype=np.float64)
    t = ct.c_uint64()
    _check(lib.sbqa_submit(srv.ptr, ct.byref(c), _p(hd), N, R, runs, ct.byref(schedule), ct.byref(t)))
    srv.shapes[t.value] = (runs, N)
    return t.value


def sbqa_poll(srv: Server, ticket: int):
    """None while pending, else (energies, spins, latency_s)."""
    runs, N = srv.shapes[ticket]
    E = np.empty(runs)
    s = np.empty((runs, N), dtype=np.int8)
    lat = ct.c_double()
    st = lib.sbqa_poll(srv.ptr, ticket, _p(E), _p(s), ct.byref(lat))
    if st == EAGAIN:
        return None
    _check(st)
    del srv.shapes[ticket]
    return E, s, lat.value


def sbqa_server_stats(srv: Server):
    done = ct.c_uint64()
    upd = ct.c_double()
    busy = ct.c_double()
    _check(lib.sbqa_server_stats(srv.ptr, ct.byref(done), ct.byref(upd), ct.byref(busy)))
    return {"completed": done.value, "updates": upd.value, "busy_s": busy.value}


def sbqa_server_destroy(srv: Server) -> None:
    if srv.ptr:
        lib.sbqa_server_destroy(srv.ptr)
        srv.ptr = None


__all__ = [n for n in dir() if n.startswith("sbqa_")]
