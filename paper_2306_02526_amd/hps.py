"""Thin ctypes binding of libhps.so (argument marshalling only).

Every function here has the name of the C entry point it calls (include/hps.h).
Device arrays are PyTorch CUDA float64 tensors; the library runs every step of the
build and of the solves in its own HIP kernels.  There is no fallback: if the
library is missing or no GPU is present the calls raise.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HPS_LIB", os.path.join(HERE, "libhps.so"))

HPS_FP64 = 0
HPS_FP32_IR = 1
HPS_WIDE_TILES = 2
HPS_UNIFORM_COEFFS = 4
HPS_IR_STRICT = 8
HPS_TEST_FP32_SKEW = 16
HPS_AUTOTUNE = 32
ERRORS = {-1: "HPS_EINVAL", -2: "HPS_ENOMEM", -3: "HPS_EDEVICE", -4: "HPS_ESINGULAR",
          -5: "HPS_ENOTCONVERGED", -6: "HPS_EBUSY"}

# every entry point declared in include/hps.h, include/hps_batch.h and include/hps_serve.h
EXPORTED = ["hps_last_error", "hps_num_nodes", "hps_nodes", "hps_build", "hps_op_bytes",
            "hps_solve", "hps_solve_noalloc", "hps_free", "hps_build_complex", "hps_profile_enable", "hps_profile_read", "ark_create", "ark_step", "ark_info", "ark_stage_solves_per_step",
            "ark_free", "ark_step_slope", "ark_step_burgers", "hps_solve_batched", "ark_step_batched", "hps_batch_streams",
            "srv_create", "srv_submit", "srv_poll", "srv_wait", "srv_release", "srv_get_stats", "srv_destroy"]


class HPSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class HpsGrid(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double),
                ("y1", ctypes.c_double), ("n1", ctypes.c_int32), ("n2", ctypes.c_int32),
                ("p", ctypes.c_int32)]


class HpsCoeffs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("cxx", "cyy", "cx", "cy", "c0")]


class HpsInfo(ctypes.Structure):
    _fields_ = [("ir_iterations", ctypes.c_int32), ("last_correction", ctypes.c_double),
                ("fp64_fallbacks", ctypes.c_int32)]

    def as_dict(self):
        return {"ir_iterations": self.ir_iterations, "last_correction": self.last_correction,
                "fp64_fallbacks": self.fp64_fallbacks}


class ArkTableau(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int32)] + [(n, ctypes.POINTER(ctypes.c_double))
                                          for n in ("A", "b", "c", "Ahat", "bhat")]


class ArkG(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("g0", ctypes.c_double), ("g1", ctypes.c_double),
                ("g2", ctypes.c_double), ("g3", ctypes.c_double)]


class SrvConfig(ctypes.Structure):
    _fields_ = [("cache_bytes", ctypes.c_int64), ("max_active", ctypes.c_int32), ("max_queued", ctypes.c_int32)]


class SrvJob(ctypes.Structure):
    _fields_ = [("grid", HpsGrid), ("coef_key", ctypes.c_uint64), ("coeffs", HpsCoeffs),
                ("flags", ctypes.c_int32), ("tab", ArkTableau), ("dt", ctypes.c_double), ("g", ArkG),
                ("t0", ctypes.c_double), ("steps", ctypes.c_int32), ("u", ctypes.c_void_p),
                ("q_space", ctypes.c_void_p), ("q_amp", ctypes.c_double), ("q_rate", ctypes.c_double)]


class SrvStatus(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("error", ctypes.c_int32), ("steps_done", ctypes.c_int32),
                ("cache_hit", ctypes.c_int32), ("submit_s", ctypes.c_double), ("start_s", ctypes.c_double),
                ("finish_s", ctypes.c_double)]


class SrvStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "failed", "builds", "cache_hits",
                                              "evictions", "cached_ops", "cached_bytes", "iterations",
                                              "job_steps", "context_bytes", "waits")]


SRV_QUEUED, SRV_ACTIVE, SRV_DONE, SRV_FAILED = 0, 1, 2, 3

_lib = None


def lib():
    """Load libhps.so (built by paper_2306_02526_amd.build_lib)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2306_02526_amd.build_lib`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.hps_last_error.restype = ctypes.c_char_p
    L.hps_last_error.argtypes = []
    L.hps_num_nodes.restype = i64
    L.hps_num_nodes.argtypes = [P(HpsGrid), P(i64), P(i64), P(i64)]
    L.hps_nodes.restype = i32
    L.hps_nodes.argtypes = [P(HpsGrid), P(dbl), P(dbl)]
    L.hps_build.restype = i32
    L.hps_build.argtypes = [P(HpsGrid), P(HpsCoeffs), dbl, i32, vp, P(vp)]
    L.hps_build_complex.restype = i32
    L.hps_build_complex.argtypes = [P(HpsGrid), P(HpsCoeffs), P(HpsCoeffs), dbl, i32, vp, P(vp)]
    L.hps_op_bytes.restype = i64
    L.hps_op_bytes.argtypes = [vp, P(i64)]
    L.hps_solve.restype = i32
    L.hps_solve.argtypes = [vp, i32, vp, vp, vp, vp, vp, P(HpsInfo)]
    L.hps_solve_noalloc.restype = i32
    L.hps_solve_noalloc.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    L.hps_free.restype = None
    L.hps_free.argtypes = [vp]
    L.hps_profile_enable.restype = i32
    L.hps_profile_enable.argtypes = [vp, i32]
    L.hps_profile_read.restype = i32
    L.hps_profile_read.argtypes = [vp, i32, P(ctypes.c_char_p), P(i64), P(dbl)]
    L.ark_create.restype = i32
    L.ark_create.argtypes = [vp, P(ArkTableau), dbl, P(ArkG), P(vp)]
    L.ark_step.restype = i32
    L.ark_step.argtypes = [vp, dbl, vp, vp, vp, P(dbl), vp, vp]
    L.ark_step_slope.restype = i32
    L.ark_step_slope.argtypes = [vp, dbl, vp, vp, vp, P(dbl), vp, vp]
    L.ark_step_burgers.restype = i32
    L.ark_step_burgers.argtypes = [vp, vp, dbl, vp, vp, vp, vp, vp]
    L.ark_stage_solves_per_step.restype = i32
    L.ark_stage_solves_per_step.argtypes = [vp]
    L.ark_info.restype = i32
    L.ark_info.argtypes = [vp, P(HpsInfo)]
    L.ark_free.restype = None
    L.ark_free.argtypes = [vp]
    L.hps_solve_batched.restype = i32
    L.hps_solve_batched.argtypes = [P(vp), i32, P(vp), P(vp), P(vp), P(vp), vp, P(HpsInfo)]
    L.ark_step_batched.restype = i32
    L.ark_step_batched.argtypes = [P(vp), i32, P(dbl), P(vp), P(vp), P(vp), P(vp), P(vp), vp]
    L.hps_batch_streams.restype = i32
    L.hps_batch_streams.argtypes = []
    L.srv_create.restype = i32
    L.srv_create.argtypes = [P(SrvConfig), P(vp)]
    L.srv_submit.restype = i32
    L.srv_submit.argtypes = [vp, P(SrvJob), vp, P(i64)]
    L.srv_poll.restype = i32
    L.srv_poll.argtypes = [vp, i64, P(SrvStatus)]
    L.srv_wait.restype = i32
    L.srv_wait.argtypes = [vp, i64, P(SrvStatus)]
    L.srv_release.restype = i32
    L.srv_release.argtypes = [vp, i64]
    L.srv_get_stats.restype = i32
    L.srv_get_stats.argtypes = [vp, P(SrvStats)]
    L.srv_destroy.restype = None
    L.srv_destroy.argtypes = [vp]
    _lib = L
    return L


def _check(rc):
    if rc < 0:
        raise HPSError(rc, lib().hps_last_error().decode())
    return rc


def hps_last_error():
    return lib().hps_last_error().decode()


def make_grid(x0, x1, y0, y1, n1, n2, p):
    return HpsGrid(float(x0), float(x1), float(y0), float(y1), int(n1), int(n2), int(p))


def hps_num_nodes(grid):
    """(N, n_int, n_iface, n_bdry)"""
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    N = _check(lib().hps_num_nodes(ctypes.byref(grid), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return int(N), a.value, b.value, c.value


def hps_nodes(grid):
    N = hps_num_nodes(grid)[0]
    x = np.empty(N)
    y = np.empty(N)
    P = ctypes.POINTER(ctypes.c_double)
    _check(lib().hps_nodes(ctypes.byref(grid), x.ctypes.data_as(P), y.ctypes.data_as(P)))
    return x, y


def _dptr(t, n=None, name="array"):
    """Device pointer of a contiguous float64 CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


class HpsOp:
    """Owns an hps_op handle (freed with hps_free)."""

    def __init__(self, handle, grid, gamma_dt, flags, sizes, keep, ncomp=1):
        self.handle = handle
        self.grid = grid
        self.gamma_dt = gamma_dt
        self.flags = flags
        self.ncomp = ncomp        # 2: complex operator, vectors as [real plane, imaginary plane]
        self.N, self.n_int, self.n_iface, self.n_bdry = sizes
        self._keep = keep

    def bytes(self):
        ob = ctypes.c_int64()
        tot = _check(lib().hps_op_bytes(self.handle, ctypes.byref(ob)))
        return int(tot), ob.value

    def free(self):
        if self.handle:
            lib().hps_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def hps_profile_enable(op, enable=True):
    _check(lib().hps_profile_enable(op.handle, 1 if enable else 0))


def hps_profile_read(op):
    """{kernel family: (launches, total_ms)} recorded since the last read."""
    m = 32
    names = (ctypes.c_char_p * m)()
    cnt = (ctypes.c_int64 * m)()
    ms = (ctypes.c_double * m)()
    n = _check(lib().hps_profile_read(op.handle, m, names, cnt, ms))
    return {names[i].decode(): (int(cnt[i]), float(ms[i])) for i in range(min(n, m))}


def hps_build(grid, coeffs, gamma_dt, flags=HPS_FP64, stream=None):
    """coeffs: dict with any of cxx, cyy, cx, cy, c0 -> float64 CUDA tensors of n_int."""
    sizes = hps_num_nodes(grid)
    n_int = sizes[1]
    keep = {k: v for k, v in coeffs.items() if v is not None}
    c = HpsCoeffs(*[_dptr(coeffs.get(k), n_int, k) for k in ("cxx", "cyy", "cx", "cy", "c0")])
    h = ctypes.c_void_p()
    _check(lib().hps_build(ctypes.byref(grid), ctypes.byref(c), float(gamma_dt), int(flags),
                           _stream(stream), ctypes.byref(h)))
    return HpsOp(h, grid, float(gamma_dt), flags, sizes, keep)


def hps_build_complex(grid, coeffs_re, coeffs_im, gamma_dt, flags=HPS_FP64, stream=None):
    """Complex coefficients: coeffs_re / coeffs_im dicts of float64 CUDA tensors (real and
    imaginary parts, any of cxx, cyy, cx, cy, c0)."""
    sizes = hps_num_nodes(grid)
    n_int = sizes[1]
    keep = [v for d in (coeffs_re, coeffs_im) for v in d.values() if v is not None]
    cr = HpsCoeffs(*[_dptr(coeffs_re.get(k), n_int, k) for k in ("cxx", "cyy", "cx", "cy", "c0")])
    ci = HpsCoeffs(*[_dptr(coeffs_im.get(k), n_int, k) for k in ("cxx", "cyy", "cx", "cy", "c0")])
    h = ctypes.c_void_p()
    _check(lib().hps_build_complex(ctypes.byref(grid), ctypes.byref(cr), ctypes.byref(ci), float(gamma_dt),
                                   int(flags), _stream(stream), ctypes.byref(h)))
    return HpsOp(h, grid, float(gamma_dt), flags, sizes, keep, ncomp=2)


HPS_NOALLOC_SCRATCH_BYTES = 32 << 20   # the fixed device array of hps_solve_noalloc


def hps_solve_noalloc(op, body, dirichlet=None, jump=None, u=None, stream=None):
    """hps_solve without allocation in the library (FP64 real operators): its intermediate
    data go to the library's fixed per-GPU scratch array.  body [nrhs, n_int] or [n_int];
    u (output) is allocated here by torch unless given."""
    import torch
    squeeze = body.dim() == 1
    nrhs = 1 if squeeze else body.shape[0]
    if u is None:
        u = torch.empty((op.N,) if squeeze else (nrhs, op.N), dtype=torch.float64, device=body.device)
    _check(lib().hps_solve_noalloc(op.handle, nrhs, _dptr(body, nrhs * op.n_int, "body"),
                                   _dptr(dirichlet, nrhs * op.n_bdry, "dirichlet"),
                                   _dptr(jump, nrhs * op.n_iface, "jump"), _dptr(u, nrhs * op.N, "u"),
                                   _stream(stream)))
    return u


def hps_solve_complex(op, body, dirichlet=None, jump=None, u=None, stream=None):
    """Complex operator, one right-hand side: body [2, n_int] (real, imaginary plane),
    dirichlet [2, n_bdry], jump [2, n_iface]; returns u [2, N]."""
    import torch
    if op.ncomp != 2:
        raise ValueError("hps_solve_complex needs an operator from hps_build_complex")
    if u is None:
        u = torch.empty((2, op.N), dtype=torch.float64, device=body.device)
    _check(lib().hps_solve(op.handle, 1, _dptr(body, 2 * op.n_int, "body"), _dptr(dirichlet, 2 * op.n_bdry, "dirichlet"),
                           _dptr(jump, 2 * op.n_iface, "jump"), _dptr(u, 2 * op.N, "u"), _stream(stream), None))
    return u


def hps_solve(op, body, dirichlet=None, jump=None, u=None, stream=None, info=False):
    """Solve (I - gamma_dt L) u = body; body [nrhs, n_int] or [n_int]. Returns u."""
    import torch
    squeeze = body.dim() == 1
    nrhs = 1 if squeeze else body.shape[0]
    if u is None:
        u = torch.empty((op.N,) if squeeze else (nrhs, op.N), dtype=torch.float64, device=body.device)
    inf = HpsInfo()
    _check(lib().hps_solve(op.handle, nrhs, _dptr(body, nrhs * op.n_int, "body"),
                           _dptr(dirichlet, nrhs * op.n_bdry, "dirichlet"),
                           _dptr(jump, nrhs * op.n_iface, "jump"), _dptr(u, nrhs * op.N, "u"),
                           _stream(stream), ctypes.byref(inf) if info else None))
    if info:
        return u, inf.as_dict()
    return u


class ArkCtx:
    def __init__(self, handle, op, s):
        self.handle = handle
        self.op = op
        self.s = s

    def free(self):
        if self.handle:
            lib().ark_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def ark_create(op, tableau, dt, g=None):
    """tableau: dict with s, A (s x s), b, c, Ahat, bhat.  g: None or (g0, g1, g2, g3): the
    polynomial g0 + g1 u + g2 u^2 + g3 u^3, or for a complex operator the NLS form
    (g0 + i g1) u + (g2 + i g3) |u|^2 u."""
    s = int(tableau["s"])
    arrs = {k: np.ascontiguousarray(np.asarray(tableau[k], dtype=np.float64).ravel())
            for k in ("A", "b", "c", "Ahat", "bhat")}
    P = ctypes.POINTER(ctypes.c_double)
    tab = ArkTableau(s, *[arrs[k].ctypes.data_as(P) for k in ("A", "b", "c", "Ahat", "bhat")])
    kind = 2 if getattr(op, "ncomp", 1) == 2 else 1
    gg = ArkG(0, 0.0, 0.0, 0.0, 0.0) if g is None else ArkG(kind, *[float(v) for v in g])
    h = ctypes.c_void_p()
    _check(lib().ark_create(op.handle, ctypes.byref(tab), float(dt), ctypes.byref(gg), ctypes.byref(h)))
    return ArkCtx(h, op, s)


def ark_step(ctx, t, u, q_stages=None, q_space=None, q_time=None, f_stages=None, stream=None):
    op, s = ctx.op, ctx.s
    qt = None
    if q_time is not None:
        qt_arr = np.ascontiguousarray(np.asarray(q_time, dtype=np.float64))
        if qt_arr.size != s:
            raise ValueError("q_time needs one value per stage")
        qt = qt_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    m = getattr(op, "ncomp", 1)   # complex: u [2, N], f_stages [s + 1, 2, n_bdry]
    _check(lib().ark_step(ctx.handle, float(t), _dptr(u, m * op.N, "u"),
                          _dptr(q_stages, s * op.n_int, "q_stages"), _dptr(q_space, op.n_int, "q_space"),
                          qt, _dptr(f_stages, (s + 1) * m * op.n_bdry, "f_stages"), _stream(stream)))
    return u


def ark_step_slope(ctx, t, u, q_stages=None, q_space=None, q_time=None, fdot_stages=None, stream=None):
    """One slope-formulation step (flux-jump penalised); fdot_stages [s][n_bdry] or None."""
    op, s = ctx.op, ctx.s
    qt = None
    if q_time is not None:
        qt_arr = np.ascontiguousarray(np.asarray(q_time, dtype=np.float64))
        if qt_arr.size != s:
            raise ValueError("q_time needs one value per stage")
        qt = qt_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(lib().ark_step_slope(ctx.handle, float(t), _dptr(u, op.N, "u"),
                                _dptr(q_stages, s * op.n_int, "q_stages"), _dptr(q_space, op.n_int, "q_space"),
                                qt, _dptr(fdot_stages, s * op.n_bdry, "fdot_stages"), _stream(stream)))
    return u


def ark_step_burgers(cu, cv, t, u, v, fu_stages=None, fv_stages=None, stream=None):
    """One step of the 2-D Burgers system on the contexts cu, cv of one operator, in place on
    u and v; fu_stages, fv_stages: Dirichlet data [s+1][n_bdry] of each component or None."""
    op, s = cu.op, cu.s
    _check(lib().ark_step_burgers(cu.handle, cv.handle, float(t), _dptr(u, op.N, "u"), _dptr(v, op.N, "v"),
                                  _dptr(fu_stages, (s + 1) * op.n_bdry, "fu_stages"),
                                  _dptr(fv_stages, (s + 1) * op.n_bdry, "fv_stages"), _stream(stream)))
    return u, v


def ark_info(ctx):
    """Refinement record of the last ark_step (FP32_IR operators; zeros for FP64)."""
    inf = HpsInfo()
    _check(lib().ark_info(ctx.handle, ctypes.byref(inf)))
    return inf.as_dict()


def ark_stage_solves_per_step(ctx):
    return _check(lib().ark_stage_solves_per_step(ctx.handle))


# ---------------------------------------------------------------------------------------
# batched entry points (include/hps_batch.h)
# ---------------------------------------------------------------------------------------
def _ptr_array(items, sizes, name, required=False):
    """Host array of device pointers (None for an absent list or entry)."""
    if items is None:
        if required:
            raise ValueError(f"{name} is required")
        return None
    if len(items) != len(sizes):
        raise ValueError(f"{name} needs one entry per problem")
    arr = (ctypes.c_void_p * len(items))()
    for b, (t, n) in enumerate(zip(items, sizes)):
        if t is None and required:
            raise ValueError(f"{name}[{b}] is required")
        arr[b] = None if t is None else _dptr(t, n, f"{name}[{b}]").value
    return arr


def hps_batch_streams():
    return lib().hps_batch_streams()


def hps_solve_batched(ops, body, dirichlet=None, jump=None, u=None, stream=None, info=False):
    """One right-hand side per problem: body[b] [n_int(b)] -> u[b] [N(b)] (list of tensors)."""
    import torch
    nb = len(ops)
    if len(body) != nb or any(t is None for t in body):
        raise ValueError("body needs one tensor per problem")
    if u is None:
        u = [torch.empty(op.N, dtype=torch.float64, device=body[b].device) for b, op in enumerate(ops)]
    opa = (ctypes.c_void_p * nb)(*[op.handle for op in ops])
    inf = (HpsInfo * nb)() if info else None
    _check(lib().hps_solve_batched(opa, nb, _ptr_array(body, [o.n_int for o in ops], "body", True),
                                   _ptr_array(dirichlet, [o.n_bdry for o in ops], "dirichlet"),
                                   _ptr_array(jump, [o.n_iface for o in ops], "jump"),
                                   _ptr_array(u, [o.N for o in ops], "u", True), _stream(stream), inf))
    if info:
        return u, [i.as_dict() for i in inf]
    return u


def ark_step_batched(ctxs, t, u, q_stages=None, q_space=None, q_time=None, f_stages=None, stream=None):
    """One step of every problem: t list of floats, u list of [N(b)] tensors (in place)."""
    nb = len(ctxs)
    ca = (ctypes.c_void_p * nb)(*[c.handle for c in ctxs])
    ta = (ctypes.c_double * nb)(*[float(v) for v in t])
    ops = [c.op for c in ctxs]
    qt = None
    keep = []
    if q_time is not None:
        qt = (ctypes.c_void_p * nb)()
        for b, v in enumerate(q_time):
            if v is None:
                continue
            arr = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
            if arr.size != ctxs[b].s:
                raise ValueError(f"q_time[{b}] needs one value per stage")
            keep.append(arr)
            qt[b] = arr.ctypes.data
    _check(lib().ark_step_batched(ca, nb, ta, _ptr_array(u, [o.N for o in ops], "u", True),
                                  _ptr_array(q_stages, [c.s * c.op.n_int for c in ctxs], "q_stages"),
                                  _ptr_array(q_space, [o.n_int for o in ops], "q_space"), qt,
                                  _ptr_array(f_stages, [(c.s + 1) * c.op.n_bdry for c in ctxs], "f_stages"),
                                  _stream(stream)))
    return u


# ---------------------------------------------------------------------------------------
# time-stepping server (include/hps_serve.h)
# ---------------------------------------------------------------------------------------
def _status_dict(st):
    return {"state": st.state, "error": st.error, "steps_done": st.steps_done, "cache_hit": st.cache_hit,
            "submit_s": st.submit_s, "start_s": st.start_s, "finish_s": st.finish_s}


class Server:
    """Owns an srv_server handle (srv_destroy drains it).  Keeps every array of a job
    alive until the job is released."""

    def __init__(self, cache_bytes=0, max_active=0, max_queued=0):
        h = ctypes.c_void_p()
        cfg = SrvConfig(int(cache_bytes), int(max_active), int(max_queued))
        _check(lib().srv_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, grid, coef_key, coeffs, tableau, dt, u, steps, t0=0.0, flags=HPS_FP64, g=None,
               q_space=None, q_amp=0.0, q_rate=0.0, stream=None):
        """coeffs: dict of float64 CUDA tensors [n_int]; u: float64 CUDA tensor [N] (in/out)."""
        N, n_int, _, _ = hps_num_nodes(grid)
        s = int(tableau["s"])
        arrs = {k: np.ascontiguousarray(np.asarray(tableau[k], dtype=np.float64).ravel())
                for k in ("A", "b", "c", "Ahat", "bhat")}
        P = ctypes.POINTER(ctypes.c_double)
        tab = ArkTableau(s, *[arrs[k].ctypes.data_as(P) for k in ("A", "b", "c", "Ahat", "bhat")])
        gg = ArkG(0, 0.0, 0.0, 0.0, 0.0) if g is None else ArkG(1, *[float(v) for v in g])
        co = HpsCoeffs(*[_dptr(coeffs.get(k), n_int, k) for k in ("cxx", "cyy", "cx", "cy", "c0")])
        job = SrvJob(grid, ctypes.c_uint64(coef_key), co, int(flags), tab, float(dt), gg, float(t0),
                     int(steps), _dptr(u, N, "u"), _dptr(q_space, n_int, "q_space"), float(q_amp),
                     float(q_rate))
        jid = ctypes.c_int64()
        _check(lib().srv_submit(self.handle, ctypes.byref(job), _stream(stream), ctypes.byref(jid)))
        self._keep[jid.value] = (coeffs, u, q_space)
        return jid.value

    def poll(self, jid):
        st = SrvStatus()
        _check(lib().srv_poll(self.handle, int(jid), ctypes.byref(st)))
        return _status_dict(st)

    def wait(self, jid):
        st = SrvStatus()
        _check(lib().srv_wait(self.handle, int(jid), ctypes.byref(st)))
        return _status_dict(st)

    def release(self, jid):
        _check(lib().srv_release(self.handle, int(jid)))
        self._keep.pop(jid, None)

    def stats(self):
        st = SrvStats()
        _check(lib().srv_get_stats(self.handle, ctypes.byref(st)))
        return {n: getattr(st, n) for n, _ in SrvStats._fields_}

    def close(self):
        if self.handle:
            lib().srv_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
