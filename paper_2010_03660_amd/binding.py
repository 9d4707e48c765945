"""ctypes binding of libs7.so: argument marshalling only.

Every entry point has the name of its C function without the ``s7_`` prefix.
Arrays are torch CUDA tensors, or raw device addresses as ints.  Streams are
``torch.cuda.Stream`` objects, raw ``hipStream_t`` ints, or None for torch's
current stream.  If the library is missing, the first call raises
RuntimeError.  There is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libs7.so")

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2
EINVAL, ENOMEM, EHIP, EAGAIN, ENOTFOUND = -1, -2, -3, -4, -5
REASON_NONE, REASON_RHO_ZERO, REASON_RS_ZERO, REASON_YY_ZERO, REASON_NONFINITE = range(5)
FP32, BF16_IR, FP16_IR = 0, 1, 2
PREC_NAMES = {"fp32": FP32, "bf16_ir": BF16_IR, "fp16_ir": FP16_IR}

__all__ = [
    "Dims", "Options", "Info", "Request", "lib", "default_options", "last_error", "version",
    "stencil_apply", "workspace_bytes", "bicgstab_solve", "batched_workspace_bytes",
    "bicgstab_solve_batched", "batched_call", "queue_table_bytes", "queue_create", "queue_submit",
    "queue_poll", "queue_wait", "queue_destroy", "generate_problem", "bandwidth_probe", "S7Error",
    "stencil9_apply", "workspace_bytes_2d9", "bicgstab_solve_2d9", "generate_problem_2d9",
    "batched_workspace_bytes_2d9", "bicgstab_solve_batched_2d9", "batched_call_2d9", "Request2D9", "queue_submit_2d9", "workspace_bytes_pipelined",
    "bicgstab_solve_pipelined", "bicgstab_solve_noalloc", "NOALLOC_WS_BYTES",
    "batched_workspace_bytes_pipelined", "bicgstab_solve_batched_pipelined", "batched_pipelined_call",
    "p2_design_probe",
    "OK", "NOT_CONVERGED", "BREAKDOWN", "EINVAL", "ENOMEM", "EHIP", "EAGAIN", "ENOTFOUND",
    "REASON_NONE", "REASON_RHO_ZERO", "REASON_RS_ZERO", "REASON_YY_ZERO", "REASON_NONFINITE",
    "FP32", "BF16_IR", "FP16_IR", "PREC_NAMES", "LIB_PATH", "EXPORTS",
]


class Dims(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("jacobi", C.c_int32), ("graph_iters", C.c_int32), ("stream_blocks", C.c_int32),
                ("chunk_cells", C.c_int32), ("profile", C.c_int32), ("inner_max_iter", C.c_int32),
                ("outer_max_iter", C.c_int32), ("schedule", C.c_int32), ("tune", C.c_int32),
                ("split_cells", C.c_int32), ("inner_rtol", C.c_double), ("xcd_run", C.c_int32),
                ("lds_tile", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_iters", C.c_int32), ("status", C.c_int32),
                ("reason", C.c_int32), ("rel_res_rec", C.c_double), ("rel_res_true", C.c_double),
                ("t_ms", C.c_double), ("t_wait_ms", C.c_double), ("pass_ms", C.c_double * 4),
                ("pass_count", C.c_int32 * 4), ("schedule", C.c_int32), ("lds_tile", C.c_int32),
                ("xcd_run", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {"iters": self.iters, "outer_iters": self.outer_iters, "status": self.status,
                "reason": self.reason, "rel_res_rec": self.rel_res_rec,
                "rel_res_true": self.rel_res_true, "t_ms": self.t_ms, "t_wait_ms": self.t_wait_ms,
                "pass_ms": list(self.pass_ms), "pass_count": list(self.pass_count),
                "schedule": self.schedule, "lds_tile": self.lds_tile, "xcd_run": self.xcd_run}


class Request(C.Structure):
    _fields_ = [("d", Dims), ("coef", C.c_void_p * 7), ("b", C.c_void_p), ("x", C.c_void_p),
                ("rtol", C.c_double), ("max_iter", C.c_int32), ("prec", C.c_int32)]


class Request2D9(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("coef", C.c_void_p * 9), ("b", C.c_void_p),
                ("x", C.c_void_p), ("rtol", C.c_double), ("max_iter", C.c_int32), ("prec", C.c_int32)]


class S7Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"s7 error {code}: {msg}")
        self.code = code


_vp = C.c_void_p
EXPORTS = {
    "s7_default_options": (None, [C.POINTER(Options)]),
    "s7_last_error": (C.c_char_p, []),
    "s7_version": (C.c_int32, []),
    "s7_stencil_apply": (C.c_int, [Dims, C.POINTER(_vp), _vp, _vp, _vp]),
    "s7_workspace_bytes": (C.c_size_t, [Dims, C.c_int32, C.POINTER(Options)]),
    "s7_bicgstab_solve": (C.c_int, [Dims, C.POINTER(_vp), _vp, _vp, C.c_double, C.c_int32, C.c_int32,
                                    _vp, C.c_size_t, C.POINTER(Options), C.POINTER(Info), _vp]),
    "s7_batched_workspace_bytes": (C.c_size_t, [C.c_int32, C.POINTER(Dims), C.c_int32,
                                                C.POINTER(Options)]),
    "s7_batched_workspace_bytes_pipelined": (C.c_size_t, [C.c_int32, C.POINTER(Dims), C.POINTER(Options)]),
    "s7_bicgstab_solve_batched_pipelined": (C.c_int, [C.c_int32, C.POINTER(Dims), C.POINTER(_vp),
                                                      C.POINTER(_vp), C.POINTER(_vp),
                                                      C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                                      _vp, C.c_size_t, C.POINTER(Options), C.POINTER(Info),
                                                      _vp]),
    "s7_p2_design_part_bytes": (C.c_size_t, [C.c_int32, C.c_int32, Dims]),
    "s7_p2_design_probe": (C.c_int, [C.c_int32, C.c_int32, Dims, C.POINTER(_vp), _vp, _vp, _vp, C.c_float, _vp,
                                     _vp, C.c_size_t, C.c_int32, C.POINTER(C.c_float), _vp]),
    "s7_bicgstab_solve_batched": (C.c_int, [C.c_int32, C.POINTER(Dims), C.POINTER(_vp),
                                            C.POINTER(_vp), C.POINTER(_vp),
                                            C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_int32,
                                            _vp, C.c_size_t, C.POINTER(Options), C.POINTER(Info),
                                            _vp]),
    "s7_queue_table_bytes": (C.c_size_t, []),
    "s7_queue_create": (C.c_int, [C.POINTER(_vp), _vp, C.c_size_t, C.POINTER(Options)]),
    "s7_queue_submit": (C.c_int, [_vp, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "s7_queue_poll": (C.c_int, [_vp, C.c_uint64, C.POINTER(Info)]),
    "s7_queue_wait": (C.c_int, [_vp, C.c_uint64, C.POINTER(Info)]),
    "s7_queue_destroy": (C.c_int, [_vp]),
    "s7_generate_problem": (C.c_int, [Dims, C.c_uint64, C.c_int32, C.POINTER(_vp), _vp, _vp, _vp]),
    "s7_bandwidth_probe": (C.c_int, [C.c_int32, C.c_int32, _vp, _vp, _vp, C.c_size_t, C.c_int32, _vp]),
    "s7_stencil9_apply": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(_vp), _vp, _vp, _vp]),
    "s7_workspace_bytes_2d9": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(Options)]),
    "s7_bicgstab_solve_2d9": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(_vp), _vp, _vp, C.c_double,
                                        C.c_int32, C.c_int32, _vp, C.c_size_t, C.POINTER(Options),
                                        C.POINTER(Info), _vp]),
    "s7_generate_problem_2d9": (C.c_int, [C.c_int32, C.c_int32, C.c_uint64, C.POINTER(_vp), _vp, _vp, _vp]),
    "s7_workspace_bytes_pipelined": (C.c_size_t, [Dims, C.POINTER(Options)]),
    "s7_bicgstab_solve_pipelined": (C.c_int, [Dims, C.POINTER(_vp), _vp, _vp, C.c_double, C.c_int32, _vp,
                                              C.c_size_t, C.POINTER(Options), C.POINTER(Info), _vp]),
    "s7_queue_submit_2d9": (C.c_int, [_vp, C.POINTER(Request2D9), C.POINTER(C.c_uint64)]),
    "s7_bicgstab_solve_noalloc": (C.c_int, [Dims, C.POINTER(_vp), _vp, _vp, C.c_double, C.c_int32,
                                            C.POINTER(Options), C.POINTER(Info), _vp]),
    "s7_batched_workspace_bytes_2d9": (C.c_size_t, [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                                    C.c_int32, C.POINTER(Options)]),
    "s7_bicgstab_solve_batched_2d9": (C.c_int, [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                                C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp),
                                                C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_int32,
                                                _vp, C.c_size_t, C.POINTER(Options), C.POINTER(Info), _vp]),
}

_lib = None


def lib():
    """The loaded library.  Raises RuntimeError if libs7.so is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2010_03660_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().s7_last_error().decode()


def version() -> int:
    return lib().s7_version()


def default_options(**kw) -> Options:
    o = Options()
    lib().s7_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(t) -> int:
    if t is None:
        return 0
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dims(d) -> Dims:
    return d if isinstance(d, Dims) else Dims(*[int(v) for v in d])


def _coef(coef: Sequence) -> C.Array:
    if len(coef) != 7:
        raise ValueError("need 7 coefficient arrays: diag, xm, xp, ym, yp, zm, zp")
    return (_vp * 7)(*[_ptr(c) for c in coef])


def _check(rc: int, allow=(OK, NOT_CONVERGED, BREAKDOWN)) -> int:
    if rc not in allow:
        raise S7Error(rc, last_error())
    return rc


def stencil_apply(dims, coef, v, u, stream=None) -> None:
    _check(lib().s7_stencil_apply(_dims(dims), _coef(coef), _ptr(v), _ptr(u), _stream(stream)),
           allow=(OK,))


def workspace_bytes(dims, prec=FP32, opt: Options | None = None) -> int:
    return int(lib().s7_workspace_bytes(_dims(dims), int(prec), C.byref(opt) if opt else None))


def _workspace(nbytes: int, ws):
    if ws is not None:
        return ws
    import torch
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")


def bicgstab_solve(dims, coef, b, x, rtol, max_iter, prec=FP32, ws=None,
                   opt: Options | None = None, stream=None) -> Info:
    """Solves A x = b in place in x (x0 on entry).  Returns the Info record; raises on error codes < 0."""
    info = Info()
    nbytes = workspace_bytes(dims, prec, opt)
    ws = _workspace(nbytes, ws)
    wsb = ws.numel() * ws.element_size() if not isinstance(ws, int) else nbytes
    rc = lib().s7_bicgstab_solve(_dims(dims), _coef(coef), _ptr(b), _ptr(x), float(rtol),
                                 int(max_iter), int(prec), _ptr(ws), wsb,
                                 C.byref(opt) if opt else None, C.byref(info), _stream(stream))
    _check(rc)
    return info


NOALLOC_WS_BYTES = 64 << 20  # S7_NOALLOC_WS_BYTES


def bicgstab_solve_noalloc(dims, coef, b, x, rtol, max_iter, opt: Options | None = None,
                           stream=None) -> Info:
    """FP32 solve in place in x with the library's fixed per-GPU workspace: nothing is
    allocated.  Returns the Info record; raises on error codes < 0."""
    info = Info()
    rc = lib().s7_bicgstab_solve_noalloc(_dims(dims), _coef(coef), _ptr(b), _ptr(x), float(rtol),
                                         int(max_iter), C.byref(opt) if opt else None,
                                         C.byref(info), _stream(stream))
    _check(rc)
    return info


def batched_workspace_bytes(dims_list, prec=FP32, opt: Options | None = None) -> int:
    n = len(dims_list)
    arr = (Dims * n)(*[_dims(d) for d in dims_list])
    return int(lib().s7_batched_workspace_bytes(n, arr, int(prec), C.byref(opt) if opt else None))


def batched_call(dims_list, coefs, bs, xs, rtols, max_iters, prec=FP32, ws=None,
                 opt: Options | None = None, stream=None):
    """Marshals the arguments of s7_bicgstab_solve_batched once and returns a function
    that makes the call and returns (status, [Info]).  The arrays must stay alive and
    in place while the function is used (for callers that repeat a batch)."""
    n = len(dims_list)
    arr = (Dims * n)(*[_dims(d) for d in dims_list])
    cp = (_vp * (7 * n))(*[_ptr(c) for cs in coefs for c in cs])
    bp = (_vp * n)(*[_ptr(b) for b in bs])
    xp = (_vp * n)(*[_ptr(x) for x in xs])
    rt = (C.c_double * n)(*[float(r) for r in rtols])
    mi = (C.c_int32 * n)(*[int(m) for m in max_iters])
    infos = (Info * n)()
    nbytes = batched_workspace_bytes(dims_list, prec, opt)
    ws = _workspace(nbytes, ws)
    wsb = ws.numel() * ws.element_size() if not isinstance(ws, int) else nbytes
    fn, wsp, ob, st = lib().s7_bicgstab_solve_batched, _ptr(ws), C.byref(opt) if opt else None, _stream(stream)

    def call():
        rc = fn(n, arr, cp, bp, xp, rt, mi, int(prec), wsp, wsb, ob, infos, st)
        _check(rc)
        return rc, list(infos)
    call.keep = (arr, cp, bp, xp, rt, mi, infos, ws, opt)
    return call


def bicgstab_solve_batched(dims_list, coefs, bs, xs, rtols, max_iters, prec=FP32, ws=None,
                           opt: Options | None = None, stream=None):
    """Solves len(dims_list) systems in one persistent launch.  Returns (status, [Info])."""
    return batched_call(dims_list, coefs, bs, xs, rtols, max_iters, prec, ws, opt, stream)()


def queue_table_bytes() -> int:
    return int(lib().s7_queue_table_bytes())


def queue_create(arena, arena_bytes: int | None = None, opt: Options | None = None) -> int:
    q = _vp()
    nbytes = arena_bytes if arena_bytes is not None else arena.numel() * arena.element_size()
    _check(lib().s7_queue_create(C.byref(q), _ptr(arena), nbytes, C.byref(opt) if opt else None),
           allow=(OK,))
    return q.value


def queue_submit(q: int, dims, coef, b, x, rtol, max_iter, prec=FP32) -> int:
    req = Request(_dims(dims), (_vp * 7)(*[_ptr(c) for c in coef]), _ptr(b), _ptr(x), float(rtol),
                  int(max_iter), int(prec))
    t = C.c_uint64()
    _check(lib().s7_queue_submit(q, C.byref(req), C.byref(t)), allow=(OK,))
    return t.value


def queue_poll(q: int, ticket: int):
    """(status or EAGAIN, Info)."""
    info = Info()
    rc = lib().s7_queue_poll(q, ticket, C.byref(info))
    _check(rc, allow=(OK, NOT_CONVERGED, BREAKDOWN, EAGAIN))
    return rc, info


def queue_wait(q: int, ticket: int):
    info = Info()
    rc = lib().s7_queue_wait(q, ticket, C.byref(info))
    _check(rc)
    return rc, info


def queue_destroy(q: int) -> None:
    _check(lib().s7_queue_destroy(q), allow=(OK,))


def generate_problem(dims, seed: int, recipe: int, coef=None, xstar=None, b=None, stream=None):
    cp = _coef(coef) if coef is not None else None
    _check(lib().s7_generate_problem(_dims(dims), int(seed), int(recipe), cp, _ptr(xstar), _ptr(b),
                                     _stream(stream)), allow=(OK,))


def bandwidth_probe(kind: int, width: int, a, b, c, n: int, blocks: int, stream=None) -> None:
    _check(lib().s7_bandwidth_probe(int(kind), int(width), _ptr(a), _ptr(b), _ptr(c), int(n),
                                    int(blocks), _stream(stream)), allow=(OK,))


# ---- the 2D 9-point operator: coefficients (diag, w, e, s, n, sw, se, nw, ne)
def _coef9(coef: Sequence) -> C.Array:
    if len(coef) != 9:
        raise ValueError("need 9 coefficient arrays: diag, w, e, s, n, sw, se, nw, ne")
    return (_vp * 9)(*[_ptr(c) for c in coef])


def stencil9_apply(nx: int, ny: int, coef, v, u, stream=None) -> None:
    _check(lib().s7_stencil9_apply(int(nx), int(ny), _coef9(coef), _ptr(v), _ptr(u), _stream(stream)),
           allow=(OK,))


def workspace_bytes_2d9(nx: int, ny: int, prec=FP32, opt: Options | None = None) -> int:
    return int(lib().s7_workspace_bytes_2d9(int(nx), int(ny), int(prec), C.byref(opt) if opt else None))


def bicgstab_solve_2d9(nx: int, ny: int, coef, b, x, rtol, max_iter, prec=FP32, ws=None,
                       opt: Options | None = None, stream=None) -> Info:
    """BiCGStab on the 2D 9-point system, in place in x (x0 on entry)."""
    info = Info()
    nbytes = workspace_bytes_2d9(nx, ny, prec, opt)
    ws = _workspace(nbytes, ws)
    wsb = ws.numel() * ws.element_size() if not isinstance(ws, int) else nbytes
    rc = lib().s7_bicgstab_solve_2d9(int(nx), int(ny), _coef9(coef), _ptr(b), _ptr(x), float(rtol),
                                     int(max_iter), int(prec), _ptr(ws), wsb, C.byref(opt) if opt else None,
                                     C.byref(info), _stream(stream))
    _check(rc)
    return info


def generate_problem_2d9(nx: int, ny: int, seed: int, coef=None, xstar=None, b=None, stream=None):
    cp = _coef9(coef) if coef is not None else None
    _check(lib().s7_generate_problem_2d9(int(nx), int(ny), int(seed), cp, _ptr(xstar), _ptr(b),
                                         _stream(stream)), allow=(OK,))


def _sides(meshes):
    n = len(meshes)
    return n, (C.c_int32 * n)(*[int(m[0]) for m in meshes]), (C.c_int32 * n)(*[int(m[1]) for m in meshes])


def batched_workspace_bytes_2d9(meshes, prec=FP32, opt: Options | None = None) -> int:
    """meshes: a list of (nx, ny)."""
    n, nx, ny = _sides(meshes)
    return int(lib().s7_batched_workspace_bytes_2d9(n, nx, ny, int(prec), C.byref(opt) if opt else None))


def batched_call_2d9(meshes, coefs, bs, xs, rtols, max_iters, prec=FP32, ws=None,
                     opt: Options | None = None, stream=None):
    """Marshals the arguments of s7_bicgstab_solve_batched_2d9 once and returns a
    function that makes the call and returns (status, [Info]) (see batched_call)."""
    n, nx, ny = _sides(meshes)
    if any(len(cs) != 9 for cs in coefs):
        raise ValueError("need 9 coefficient arrays per system: diag, w, e, s, n, sw, se, nw, ne")
    cp = (_vp * (9 * n))(*[_ptr(c) for cs in coefs for c in cs])
    bp = (_vp * n)(*[_ptr(b) for b in bs])
    xp = (_vp * n)(*[_ptr(x) for x in xs])
    rt = (C.c_double * n)(*[float(r) for r in rtols])
    mi = (C.c_int32 * n)(*[int(m) for m in max_iters])
    infos = (Info * n)()
    nbytes = batched_workspace_bytes_2d9(meshes, prec, opt)
    ws = _workspace(nbytes, ws)
    wsb = ws.numel() * ws.element_size() if not isinstance(ws, int) else nbytes
    fn, wsp, ob, st = lib().s7_bicgstab_solve_batched_2d9, _ptr(ws), C.byref(opt) if opt else None, _stream(stream)

    def call():
        rc = fn(n, nx, ny, cp, bp, xp, rt, mi, int(prec), wsp, wsb, ob, infos, st)
        _check(rc)
        return rc, list(infos)
    call.keep = (nx, ny, cp, bp, xp, rt, mi, infos, ws, opt)
    return call


def bicgstab_solve_batched_2d9(meshes, coefs, bs, xs, rtols, max_iters, prec=FP32, ws=None,
                               opt: Options | None = None, stream=None):
    """Solves len(meshes) 2D 9-point systems in one persistent launch; meshes is a
    list of (nx, ny), coefs a list of nine arrays each.  Returns (status, [Info])."""
    return batched_call_2d9(meshes, coefs, bs, xs, rtols, max_iters, prec, ws, opt, stream)()


def queue_submit_2d9(q: int, nx: int, ny: int, coef, b, x, rtol, max_iter, prec=FP32) -> int:
    """Queues a 2D 9-point request; coef holds nine arrays.  Returns its ticket."""
    req = Request2D9(int(nx), int(ny), _coef9(coef), _ptr(b), _ptr(x), float(rtol), int(max_iter), int(prec))
    t = C.c_uint64()
    _check(lib().s7_queue_submit_2d9(q, C.byref(req), C.byref(t)), allow=(OK,))
    return t.value


def workspace_bytes_pipelined(dims, opt: Options | None = None) -> int:
    return int(lib().s7_workspace_bytes_pipelined(_dims(dims), C.byref(opt) if opt else None))


def bicgstab_solve_pipelined(dims, coef, b, x, rtol, max_iter, ws=None, opt: Options | None = None,
                             stream=None) -> Info:
    """Pipelined BiCGStab (one reduction per iteration, residual replacement), FP32, in
    place in x (x0 on entry)."""
    info = Info()
    nbytes = workspace_bytes_pipelined(dims, opt)
    ws = _workspace(nbytes, ws)
    wsb = ws.numel() * ws.element_size() if not isinstance(ws, int) else nbytes
    rc = lib().s7_bicgstab_solve_pipelined(_dims(dims), _coef(coef), _ptr(b), _ptr(x), float(rtol), int(max_iter),
                                           _ptr(ws), wsb, C.byref(opt) if opt else None, C.byref(info),
                                           _stream(stream))
    _check(rc)
    return info


def batched_workspace_bytes_pipelined(dims_list, opt: Options | None = None) -> int:
    n = len(dims_list)
    arr = (Dims * n)(*[_dims(d) for d in dims_list])
    return int(lib().s7_batched_workspace_bytes_pipelined(n, arr, C.byref(opt) if opt else None))


def batched_pipelined_call(dims_list, coefs, bs, xs, rtols, max_iters, ws=None, opt: Options | None = None,
                           stream=None):
    """Marshals the arguments of s7_bicgstab_solve_batched_pipelined once and returns a
    function that makes the call and returns (status, [Info]) (see batched_call)."""
    n = len(dims_list)
    arr = (Dims * n)(*[_dims(d) for d in dims_list])
    cp = (_vp * (7 * n))(*[_ptr(c) for cs in coefs for c in cs])
    bp = (_vp * n)(*[_ptr(b) for b in bs])
    xp = (_vp * n)(*[_ptr(x) for x in xs])
    rt = (C.c_double * n)(*[float(r) for r in rtols])
    mi = (C.c_int32 * n)(*[int(m) for m in max_iters])
    infos = (Info * n)()
    nbytes = batched_workspace_bytes_pipelined(dims_list, opt)
    ws = _workspace(nbytes, ws)
    wsb = ws.numel() * ws.element_size() if not isinstance(ws, int) else nbytes
    fn, wsp, ob, st = lib().s7_bicgstab_solve_batched_pipelined, _ptr(ws), C.byref(opt) if opt else None, _stream(stream)

    def call():
        rc = fn(n, arr, cp, bp, xp, rt, mi, wsp, wsb, ob, infos, st)
        _check(rc)
        return rc, list(infos)
    call.keep = (arr, cp, bp, xp, rt, mi, infos, ws, opt)
    return call


def bicgstab_solve_batched_pipelined(dims_list, coefs, bs, xs, rtols, max_iters, ws=None,
                                     opt: Options | None = None, stream=None):
    """Pipelined BiCGStab for len(dims_list) systems in one persistent launch (FP32).
    Returns (status, [Info])."""
    return batched_pipelined_call(dims_list, coefs, bs, xs, rtols, max_iters, ws, opt, stream)()


def p2_design_probe(kind: int, param: int, dims, coef6, r, s, rhat, alpha: float, y, reps: int = 10,
                    part=None, stream=None):
    """Times one P2 kernel design (s7_p2_design_probe); returns (ms per launch, the five
    sums as a list).  coef6: the unit-diagonal operator's six off-diagonal arrays."""
    import torch
    d = _dims(dims)
    nbytes = int(lib().s7_p2_design_part_bytes(int(kind), int(param), d))
    if part is None:
        part = torch.empty(max(nbytes // 8, 1), dtype=torch.float64, device=r.device)
    ms = C.c_float()
    cp = (_vp * 6)(*[_ptr(c) for c in coef6])
    rc = lib().s7_p2_design_probe(int(kind), int(param), d, cp, _ptr(r), _ptr(s), _ptr(rhat), float(alpha),
                                  _ptr(y), _ptr(part), part.numel() * part.element_size(), int(reps),
                                  C.byref(ms), _stream(stream))
    _check(rc, allow=(OK,))
    sums = part[: nbytes // 8].view(-1, 5).sum(dim=0).tolist()
    return ms.value, sums
