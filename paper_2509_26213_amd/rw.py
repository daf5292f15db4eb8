"""Python binding of librw.so (argument marshalling only).

Every function here forwards to the C ABI declared in include/rw.h; all
arithmetic runs in the library's HIP kernels.  Tensors must live on the GPU;
the current torch stream is passed as the call's stream.  If the library is
missing the import of ``lib()`` raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import warnings

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librw.so")

RW_MAX_LABELS = 16
RW_OK = 0
RW_NOT_CONVERGED = 1
RW_ERR_INVALID_ARG = -1
RW_ERR_NO_SEEDS = -2
RW_ERR_SINGULAR = -3
RW_ERR_BREAKDOWN = -4
RW_ERR_NONFINITE = -5
RW_ERR_WORKSPACE = -6
RW_ERR_HIP = -7
RW_ERR_UNSUPPORTED = -8

RW_DT_U16, RW_DT_F32, RW_DT_F64 = 1, 2, 3
PREC = {"fp64": 0, "mixed": 1}

# every symbol include/rw.h declares
EXPORTS = [
    "rw_context_create", "rw_context_destroy", "rw_status_string", "rw_last_error",
    "rw_default_options", "rw_minmax", "rw_build_weights", "rw_operator_workspace_bytes",
    "rw_apply_operator", "rw_solve_workspace_bytes", "rw_solve", "rw_downsample",
    "rw_classify_bricks", "rw_bricks_workspace_bytes", "rw_solve_bricks", "rw_fill_bricks",
    "rw_backward_workspace_bytes", "rw_solve_backward", "rw_autotune", "rw_autotune_bricks",
    "rw_argmax", "rw_solve_noalloc", "rw_solve_noalloc_max_bytes", "rw_solve4d",
    "rw_solve4d_workspace_bytes", "rw_classify_bricks_sparse", "rw_seed_edit_bricks",
]


class RWError(RuntimeError):
    def __init__(self, status, detail):
        super().__init__(f"{detail} (status {status})")
        self.status = status


class Dims(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64)]


class Volume(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("dims", Dims),
                ("norm_lo", ctypes.c_double), ("norm_hi", ctypes.c_double)]


class Seeds(ctypes.Structure):
    _fields_ = [("labels", ctypes.c_void_p), ("num_labels", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("w_eps", ctypes.c_double), ("tol", ctypes.c_double),
                ("inner_tol", ctypes.c_double), ("update_delta", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("solve_all_labels", ctypes.c_int32),
                ("check_interval", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("kernel_timing", ctypes.c_int32), ("refine_mode", ctypes.c_int32),
                ("x0", ctypes.c_void_p), ("brick_voxels", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32 * RW_MAX_LABELS),
                ("label_status", ctypes.c_int32 * RW_MAX_LABELS),
                ("rel_residual", ctypes.c_double * RW_MAX_LABELS),
                ("num_solved", ctypes.c_int32), ("refinements", ctypes.c_int32),
                ("tile_by", ctypes.c_int32), ("tile_zc", ctypes.c_int32),
                ("device_ms", ctypes.c_double), ("loop_ms", ctypes.c_double),
                ("pass_ms", ctypes.c_double * 2), ("pass_launches", ctypes.c_int64 * 2),
                ("rhs_iterations", ctypes.c_int64), ("box_voxel_iterations", ctypes.c_int64),
                ("rhs_voxel_iterations", ctypes.c_int64), ("active_bricks", ctypes.c_int64),
                ("unknowns", ctypes.c_int64), ("tile_vx", ctypes.c_int32),
                ("tile_xcd", ctypes.c_int32), ("brick_blocks", ctypes.c_int32),
                ("tile_tuned", ctypes.c_int32), ("tile_by2", ctypes.c_int32),
                ("tile_zc2", ctypes.c_int32)]

    def to_dict(self):
        R = self.num_solved
        return dict(iters=list(self.iters[:R]), label_status=list(self.label_status[:R]),
                    rel_residual=list(self.rel_residual[:R]), num_solved=R,
                    refinements=self.refinements,
                    tile=dict(vx=self.tile_vx, by=self.tile_by, zc=self.tile_zc,
                              xcd=self.tile_xcd, by2=self.tile_by2, zc2=self.tile_zc2),
                    tile_tuned=bool(self.tile_tuned),
                    device_ms=self.device_ms,
                    loop_ms=self.loop_ms, pass_ms=list(self.pass_ms),
                    pass_launches=list(self.pass_launches), rhs_iterations=self.rhs_iterations,
                    box_voxel_iterations=self.box_voxel_iterations,
                    rhs_voxel_iterations=self.rhs_voxel_iterations,
                    active_bricks=self.active_bricks, unknowns=self.unknowns,
                    brick_blocks=self.brick_blocks)


class SubVolume(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("gx", ctypes.c_int32), ("gy", ctypes.c_int32),
                ("gz", ctypes.c_int32)]


class Brick(ctypes.Structure):
    _fields_ = [("ox", ctypes.c_int32), ("oy", ctypes.c_int32), ("oz", ctypes.c_int32),
                ("sx", ctypes.c_int32), ("sy", ctypes.c_int32), ("sz", ctypes.c_int32)]


_lib = None


def lib():
    """Load librw.so; raises if it was not built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built: run python -m paper_2509_26213_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    L.rw_context_create.argtypes = [ctypes.POINTER(P)]
    L.rw_context_destroy.argtypes = [P]
    L.rw_context_destroy.restype = None
    L.rw_status_string.argtypes = [I32]
    L.rw_status_string.restype = ctypes.c_char_p
    L.rw_last_error.restype = ctypes.c_char_p
    L.rw_default_options.argtypes = [ctypes.POINTER(Options)]
    L.rw_default_options.restype = None
    L.rw_minmax.argtypes = [P, ctypes.POINTER(Volume), ctypes.POINTER(D), P]
    L.rw_build_weights.argtypes = [P, ctypes.POINTER(Volume), D, D, I32, P, P,
                                   ctypes.POINTER(Seeds), P]
    L.rw_operator_workspace_bytes.argtypes = [Dims, I32]
    L.rw_operator_workspace_bytes.restype = SZ
    L.rw_apply_operator.argtypes = [P, ctypes.POINTER(Volume), ctypes.POINTER(Seeds), D, D, I32,
                                    P, P, P, SZ, P]
    L.rw_solve_workspace_bytes.argtypes = [Dims, I32, I32, I32]
    L.rw_solve_workspace_bytes.restype = SZ
    L.rw_solve.argtypes = [P, ctypes.POINTER(Volume), ctypes.POINTER(Seeds),
                           ctypes.POINTER(Options), P, P, P, SZ, ctypes.POINTER(Stats), P]
    L.rw_solve_noalloc.argtypes = [P, ctypes.POINTER(Volume), ctypes.POINTER(Seeds),
                                   ctypes.POINTER(Options), P, P, ctypes.POINTER(Stats), P]
    L.rw_solve4d_workspace_bytes.argtypes = [Dims, I32, I32, I32, I32]
    L.rw_solve4d_workspace_bytes.restype = SZ
    L.rw_solve4d.argtypes = [P, ctypes.POINTER(Volume), I32, ctypes.POINTER(Seeds),
                             ctypes.POINTER(Options), P, P, P, SZ, ctypes.POINTER(Stats), P]
    L.rw_solve_noalloc_max_bytes.argtypes = []
    L.rw_solve_noalloc_max_bytes.restype = SZ
    L.rw_downsample.argtypes = [P, ctypes.POINTER(Volume), P, I32, P, P, P]
    L.rw_classify_bricks.argtypes = [P, P, I32, Dims, I32, I32, P, Dims, ctypes.POINTER(I32),
                                     ctypes.POINTER(I32), D, D, ctypes.POINTER(Brick), P, I32,
                                     ctypes.POINTER(I32), P]
    L.rw_classify_bricks_sparse.argtypes = [P, P, I32, Dims, I32, I32, P, P, ctypes.c_int64, Dims,
                                            ctypes.POINTER(I32), ctypes.POINTER(I32), D, D,
                                            ctypes.POINTER(Brick), P, I32, ctypes.POINTER(I32), P]
    L.rw_seed_edit_bricks.argtypes = [P, P, P, Dims, P, P, I32, Dims, I32, I32,
                                      ctypes.POINTER(I32), ctypes.POINTER(I32), P,
                                      ctypes.POINTER(D), I32, ctypes.POINTER(I32), P]
    L.rw_bricks_workspace_bytes.argtypes = [ctypes.POINTER(Brick), I32, I32, I32, I32]
    L.rw_bricks_workspace_bytes.restype = SZ
    L.rw_solve_bricks.argtypes = [P, ctypes.POINTER(Volume), ctypes.POINTER(Seeds), P, I32, Dims,
                                  I32, ctypes.POINTER(Brick), ctypes.POINTER(SubVolume), I32,
                                  ctypes.POINTER(Options), P, P, P, SZ, ctypes.POINTER(Stats), P]
    L.rw_fill_bricks.argtypes = [P, P, I32, Dims, I32, I32, P, Dims, ctypes.POINTER(Brick),
                                 ctypes.POINTER(SubVolume), I32, P, P]
    L.rw_backward_workspace_bytes.argtypes = [Dims]
    L.rw_backward_workspace_bytes.restype = SZ
    L.rw_solve_backward.argtypes = [P, ctypes.POINTER(Volume), ctypes.POINTER(Seeds),
                                    ctypes.POINTER(Options), P, P, P, P, P, SZ,
                                    ctypes.POINTER(Stats), P]
    L.rw_argmax.argtypes = [P, P, I32, I32, ctypes.c_int64, P, P]
    L.rw_autotune.argtypes = [P, ctypes.POINTER(Volume), ctypes.POINTER(Seeds),
                              ctypes.POINTER(Options), P, P, SZ, ctypes.POINTER(I32), P]
    L.rw_autotune_bricks.argtypes = [P, ctypes.POINTER(Volume), ctypes.POINTER(Seeds), P, I32,
                                     Dims, I32, ctypes.POINTER(Brick), ctypes.POINTER(SubVolume),
                                     I32, ctypes.POINTER(Options), P, P, SZ, ctypes.POINTER(I32),
                                     P]
    for name in EXPORTS:
        fn = getattr(L, name)
        if fn.restype is ctypes.c_int:
            fn.restype = I32
    _lib = L
    return L


def _check(status, what="rw call"):
    if status < 0:
        detail = lib().rw_last_error().decode()
        raise RWError(status, f"{what} failed: {lib().rw_status_string(status).decode()}: {detail}")
    if status == RW_NOT_CONVERGED:
        warnings.warn(f"{what}: not converged (last iterate returned)", RuntimeWarning)
    return status


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Context:
    """Owns an rw_context (private stream, pinned polling buffer)."""

    def __init__(self):
        p = ctypes.c_void_p()
        _check(lib().rw_context_create(ctypes.byref(p)), "rw_context_create")
        self.handle = p

    def close(self):
        if self.handle:
            lib().rw_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = None


def default_context():
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context()
    return _default_ctx


def _dims(shape):
    nz, ny, nx = (int(s) for s in shape)
    return Dims(nx, ny, nz)


def make_volume(vol, lo=None, hi=None):
    """rw_volume for a device tensor (uint16 -> /65535 unless lo/hi given)."""
    if vol.dtype == torch.uint16:
        dt = RW_DT_U16
        lo = 0.0 if lo is None else lo
        hi = 65535.0 if hi is None else hi
    elif vol.dtype == torch.float32:
        dt = RW_DT_F32
    elif vol.dtype == torch.float64:
        dt = RW_DT_F64
    else:
        raise TypeError(f"unsupported volume dtype {vol.dtype}")
    if not vol.is_cuda or not vol.is_contiguous():
        raise ValueError("volume must be a contiguous GPU tensor")
    if lo is None or hi is None:
        mm = minmax(vol)
        lo = mm[0] if lo is None else lo
        hi = mm[1] if hi is None else hi
    v = Volume(_ptr(vol), dt, _dims(vol.shape), float(lo), float(hi))
    v._keep = vol
    return v


def _raw_volume(vol):
    dt = {torch.uint16: RW_DT_U16, torch.float32: RW_DT_F32, torch.float64: RW_DT_F64}[vol.dtype]
    v = Volume(_ptr(vol), dt, _dims(vol.shape), 0.0, 1.0)
    v._keep = vol
    return v


def minmax(vol, ctx=None):
    """(min, max) of a device volume, reduced by the library's kernels."""
    ctx = ctx or default_context()
    out = (ctypes.c_double * 2)()
    _check(lib().rw_minmax(ctx.handle, ctypes.byref(_raw_volume(vol)), out, _stream()), "rw_minmax")
    return float(out[0]), float(out[1])


def _seeds(labels, K):
    if labels.dtype != torch.uint8 or not labels.is_cuda or not labels.is_contiguous():
        raise ValueError("labels must be a contiguous uint8 GPU tensor")
    s = Seeds(_ptr(labels), int(K))
    s._keep = labels
    return s


def _alloc_ws(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def build_weights(vol, beta, precision="fp64", labels=None, w_eps=0.0, lo=None, hi=None,
                  ctx=None):
    """Materialised weights w[3][nz][ny][nx] (and dinv when labels are given)."""
    ctx = ctx or default_context()
    V = make_volume(vol, lo, hi)
    dt = torch.float64 if precision == "fp64" else torch.float32
    w = torch.empty((3,) + tuple(vol.shape), dtype=dt, device=vol.device)
    dinv = torch.empty(tuple(vol.shape), dtype=dt, device=vol.device) if labels is not None else None
    S = _seeds(labels, 1) if labels is not None else None
    _check(lib().rw_build_weights(ctx.handle, ctypes.byref(V), float(beta), float(w_eps),
                                  PREC[precision], _ptr(w), _ptr(dinv),
                                  ctypes.byref(S) if S is not None else None, _stream()),
           "rw_build_weights")
    return w, dinv


def apply_operator(vol, labels, p, beta, precision="fp64", w_eps=0.0, lo=None, hi=None, ctx=None):
    """q = L_U p with the CG kernel's matrix-free stencil (p zero on seeds)."""
    ctx = ctx or default_context()
    V = make_volume(vol, lo, hi)
    S = _seeds(labels, 1)
    dt = torch.float64 if precision == "fp64" else torch.float32
    p = p.to(dt).contiguous()
    q = torch.empty_like(p)
    nbytes = lib().rw_operator_workspace_bytes(_dims(vol.shape), PREC[precision])
    ws = _alloc_ws(nbytes, vol.device)
    _check(lib().rw_apply_operator(ctx.handle, ctypes.byref(V), ctypes.byref(S), float(beta),
                                   float(w_eps), PREC[precision], _ptr(p), _ptr(q), _ptr(ws),
                                   nbytes, _stream()), "rw_apply_operator")
    return q


def options(beta, tol=1e-6, precision="fp64", max_iter=20000, max_refine=5, inner_tol=1e-3,
            solve_all_labels=False, check_interval=16, use_graph=True, kernel_timing=False,
            w_eps=0.0, x0=None, refine_mode="reliable", update_delta=0.1, brick_voxels=0):
    o = Options()
    lib().rw_default_options(ctypes.byref(o))
    o.beta, o.tol, o.w_eps, o.inner_tol = float(beta), float(tol), float(w_eps), float(inner_tol)
    o.max_iter, o.max_refine = int(max_iter), int(max_refine)
    o.precision = PREC[precision]
    o.solve_all_labels = int(bool(solve_all_labels))
    o.check_interval = int(check_interval)
    o.use_graph = int(bool(use_graph))
    o.kernel_timing = int(bool(kernel_timing))
    o.refine_mode = {"reliable": 0, "restart": 1}[refine_mode]
    o.update_delta = float(update_delta)
    o.x0 = _ptr(x0) if x0 is not None else None
    o._keep = x0
    o.brick_voxels = int(brick_voxels)
    return o


def solve(vol, labels, K, beta, tol=1e-6, precision="fp64", lo=None, hi=None, argmax=True,
          ctx=None, workspace=None, return_stats=False, **kw):
    """Whole-volume random walker: probabilities [K][nz][ny][nx] (+ argmax labels).

    precision "fp64": float64 CG, float64 output; "mixed": float32 CG with
    float64 dots inside float64 refinement, float32 output.
    """
    ctx = ctx or default_context()
    V = make_volume(vol, lo, hi)
    S = _seeds(labels, K)
    x0 = kw.get("x0")
    if x0 is not None:
        kw["x0"] = x0.to(torch.float64).contiguous()
    o = options(beta, tol, precision, **kw)
    dt = torch.float64 if precision == "fp64" else torch.float32
    prob = torch.empty((K,) + tuple(vol.shape), dtype=dt, device=vol.device)
    am = torch.empty(tuple(vol.shape), dtype=torch.uint8, device=vol.device) if argmax else None
    nbytes = lib().rw_solve_workspace_bytes(_dims(vol.shape), K, o.precision, o.solve_all_labels)
    ws = workspace if workspace is not None and workspace.numel() >= nbytes else _alloc_ws(
        nbytes, vol.device)
    st = Stats()
    status = lib().rw_solve(ctx.handle, ctypes.byref(V), ctypes.byref(S), ctypes.byref(o),
                            _ptr(prob), _ptr(am), _ptr(ws), nbytes, ctypes.byref(st), _stream())
    _check(status, "rw_solve")
    out = (prob, am)
    if return_stats:
        d = st.to_dict()
        d["status"] = status
        return out + (d,)
    return out


# Time series refresh their float64 residual when ||r|| fell 2x (whole
# volumes: 10x): the time edges at a moving boundary carry weights far below
# float32's resolution next to a voxel's other weights, and the float32
# recurrence drifts from the true residual faster.  Measured (mixed, tol 1e-6)
# on 20 steps of 50x224x224: 1715 CG iterations and 1.15 s at 2x to 3.3x
# against 4802 and 3.15 s at 10x (float64: 1547, 2.33 s), a stall at 100x; on
# the paper's 200 steps: 10032 iterations (64.5 s) at 2x, 16054 at 3.3x, none
# within 20000 at 10x.
SERIES_UPDATE_DELTA = 0.5


def solve4d(vol, labels, K, beta, tol=1e-6, precision="fp64", lo=None, hi=None, argmax=True,
            ctx=None, workspace=None, return_stats=False, **kw):
    """4-D random walker of a volume time series vol [nt][nz][ny][nx] with
    seed labels of the same shape: probabilities [K][nt][nz][ny][nx] (+ the
    argmax labels).  Arguments otherwise as solve()."""
    ctx = ctx or default_context()
    if kw.get("update_delta") is None:
        kw.pop("update_delta", None)
        if vol.dim() == 4 and vol.shape[0] > 1:  # one time step keeps the 3-D default
            kw["update_delta"] = SERIES_UPDATE_DELTA
    if vol.dim() != 4 or tuple(labels.shape) != tuple(vol.shape):
        raise ValueError("vol and labels must be [nt][nz][ny][nx] of the same shape")
    nt, nz, ny, nx = (int(v) for v in vol.shape)
    V = make_volume(vol.view(nt * nz, ny, nx), lo, hi)
    V.dims = _dims(vol.shape[1:])
    S = _seeds(labels, K)
    x0 = kw.get("x0")
    if x0 is not None:
        kw["x0"] = x0.to(torch.float64).contiguous()
    o = options(beta, tol, precision, **kw)
    dt = torch.float64 if precision == "fp64" else torch.float32
    prob = torch.empty((K,) + tuple(vol.shape), dtype=dt, device=vol.device)
    am = torch.empty(tuple(vol.shape), dtype=torch.uint8, device=vol.device) if argmax else None
    nbytes = lib().rw_solve4d_workspace_bytes(_dims(vol.shape[1:]), nt, K, o.precision,
                                              o.solve_all_labels)
    ws = workspace if workspace is not None and workspace.numel() >= nbytes else _alloc_ws(
        nbytes, vol.device)
    st = Stats()
    status = lib().rw_solve4d(ctx.handle, ctypes.byref(V), nt, ctypes.byref(S), ctypes.byref(o),
                              _ptr(prob), _ptr(am), _ptr(ws), nbytes, ctypes.byref(st), _stream())
    _check(status, "rw_solve4d")
    out = (prob, am)
    if return_stats:
        d = st.to_dict()
        d["status"] = status
        return out + (d,)
    return out


def solve_noalloc(vol, labels, K, beta, prob_out, argmax_out=None, tol=1e-6, precision="fp64",
                  lo=None, hi=None, ctx=None, return_stats=False, **kw):
    """rw_solve_noalloc: the whole-volume solve with the library's static
    device scratch instead of a workspace (the caller provides the outputs:
    prob_out [K][grid], float64 for fp64, float32 for mixed; argmax_out uint8
    [grid] or None).  Needs lo and hi, or a uint16 volume, to allocate
    nothing here either."""
    ctx = ctx or default_context()
    V = make_volume(vol, lo, hi)
    S = _seeds(labels, K)
    o = options(beta, tol, precision, **kw)
    st = Stats()
    status = lib().rw_solve_noalloc(ctx.handle, ctypes.byref(V), ctypes.byref(S), ctypes.byref(o),
                                    _ptr(prob_out), _ptr(argmax_out), ctypes.byref(st), _stream())
    _check(status, "rw_solve_noalloc")
    if return_stats:
        d = st.to_dict()
        d["status"] = status
        return d
    return status


def solve_noalloc_max_bytes():
    return int(lib().rw_solve_noalloc_max_bytes())


def solve_workspace_bytes(shape, K, precision="fp64", solve_all_labels=False):
    return int(lib().rw_solve_workspace_bytes(_dims(shape), K, PREC[precision],
                                              int(bool(solve_all_labels))))


# ---------------------------------------------------------------- hierarchy

def _dt_code(t):
    return {torch.float32: RW_DT_F32, torch.float64: RW_DT_F64}[t.dtype]


def downsample(g, labels=None, lo=None, hi=None, out_dtype=torch.float32, ctx=None):
    """One LOD step: 2x2x2 means of the normalised intensities (+ coarse seeds)."""
    ctx = ctx or default_context()
    V = make_volume(g, lo, hi)
    cz, cy, cx = ((int(n) + 1) // 2 for n in g.shape)
    out = torch.empty((cz, cy, cx), dtype=out_dtype, device=g.device)
    lab_out = torch.empty((cz, cy, cx), dtype=torch.uint8, device=g.device) if labels is not None else None
    if labels is not None and (labels.dtype != torch.uint8 or not labels.is_contiguous()):
        raise ValueError("labels must be contiguous uint8")
    _check(lib().rw_downsample(ctx.handle, ctypes.byref(V), _ptr(labels), _dt_code(out), _ptr(out),
                               _ptr(lab_out), _stream()), "rw_downsample")
    return out, lab_out


def _bricks_array(bricks):
    arr = (Brick * max(len(bricks), 1))()
    for i, (o, sz) in enumerate(bricks):
        arr[i] = Brick(int(o[2]), int(o[1]), int(o[0]), int(sz[2]), int(sz[1]), int(sz[0]))
    return arr


def _from_brick(b):
    return ((b.oz, b.oy, b.ox), (b.sz, b.sy, b.sx))


def classify_bricks(coarse_prob, labels, factor, brick=(64, 64, 64), offset=(0, 0, 0),
                    lo_thr=0.02, hi_thr=0.98, ctx=None):
    """Candidate bricks (z-major grid order, (origin_zyx, size_zyx)) and their
    activity flags.  brick and offset are given (z, y, x)."""
    ctx = ctx or default_context()
    K = int(coarse_prob.shape[0])
    cd = _dims(coarse_prob.shape[1:])
    fd = _dims(labels.shape)
    bs = (ctypes.c_int32 * 3)(int(brick[2]), int(brick[1]), int(brick[0]))
    go = (ctypes.c_int32 * 3)(int(offset[2]), int(offset[1]), int(offset[0]))
    ncand = ctypes.c_int32(0)
    st = lib().rw_classify_bricks(ctx.handle, _ptr(coarse_prob), _dt_code(coarse_prob), cd, K,
                                  int(factor), _ptr(labels), fd, bs, go, float(lo_thr),
                                  float(hi_thr), None, None, 0, ctypes.byref(ncand), _stream())
    n = ncand.value
    arr = (Brick * n)()
    flags = (ctypes.c_uint8 * n)()
    _check(lib().rw_classify_bricks(ctx.handle, _ptr(coarse_prob), _dt_code(coarse_prob), cd, K,
                                    int(factor), _ptr(labels), fd, bs, go, float(lo_thr),
                                    float(hi_thr), arr, flags, n, ctypes.byref(ncand), _stream()),
           "rw_classify_bricks")
    return [_from_brick(arr[i]) for i in range(n)], [bool(flags[i]) for i in range(n)]


def classify_bricks_sparse(coarse_prob, seed_index, seed_label, fine_shape, factor,
                           brick=(64, 64, 64), offset=(0, 0, 0), lo_thr=0.02, hi_thr=0.98,
                           ctx=None):
    """classify_bricks with the seeds given as a list: seed_index (device
    int64, flat fine-grid indices) and seed_label (device uint8)."""
    ctx = ctx or default_context()
    K = int(coarse_prob.shape[0])
    cd = _dims(coarse_prob.shape[1:])
    fd = _dims(fine_shape)
    if seed_index.dtype != torch.int64 or seed_label.dtype != torch.uint8:
        raise ValueError("seed_index must be int64 and seed_label uint8")
    if seed_index.numel() != seed_label.numel():
        raise ValueError("seed_index and seed_label must have the same length")
    si, sl = seed_index.contiguous(), seed_label.contiguous()
    bs = (ctypes.c_int32 * 3)(int(brick[2]), int(brick[1]), int(brick[0]))
    go = (ctypes.c_int32 * 3)(int(offset[2]), int(offset[1]), int(offset[0]))
    ncand = ctypes.c_int32(0)
    args = (ctx.handle, _ptr(coarse_prob), _dt_code(coarse_prob), cd, K, int(factor), _ptr(si),
            _ptr(sl), int(si.numel()), fd, bs, go, float(lo_thr), float(hi_thr))
    lib().rw_classify_bricks_sparse(*args, None, None, 0, ctypes.byref(ncand), _stream())
    n = ncand.value
    arr = (Brick * n)()
    flags = (ctypes.c_uint8 * n)()
    _check(lib().rw_classify_bricks_sparse(*args, arr, flags, n, ctypes.byref(ncand), _stream()),
           "rw_classify_bricks_sparse")
    return [_from_brick(arr[i]) for i in range(n)], [bool(flags[i]) for i in range(n)]


def seed_edit_bricks(old_labels, new_labels, old_coarse, new_coarse, factor, brick=(64, 64, 64),
                     offset=(0, 0, 0), ctx=None):
    """Per candidate brick (the order of classify_bricks): whether a seed
    edit reaches it (holds or borders a changed voxel) and how far the
    coarse solution moved under it (rw_seed_edit_bricks)."""
    ctx = ctx or default_context()
    if old_coarse.dtype != new_coarse.dtype or old_coarse.shape != new_coarse.shape:
        raise ValueError("old and new coarse probabilities must match in shape and type")
    K = int(new_coarse.shape[0])
    oc, nc = old_coarse.contiguous(), new_coarse.contiguous()
    bs = (ctypes.c_int32 * 3)(int(brick[2]), int(brick[1]), int(brick[0]))
    go = (ctypes.c_int32 * 3)(int(offset[2]), int(offset[1]), int(offset[0]))
    ncand = ctypes.c_int32(0)
    args = (ctx.handle, _ptr(old_labels), _ptr(new_labels), _dims(new_labels.shape), _ptr(oc),
            _ptr(nc), _dt_code(nc), _dims(nc.shape[1:]), K, int(factor), bs, go)
    lib().rw_seed_edit_bricks(*args, None, None, 0, ctypes.byref(ncand), _stream())
    n = ncand.value
    ed = (ctypes.c_uint8 * n)()
    mv = (ctypes.c_double * n)()
    _check(lib().rw_seed_edit_bricks(*args, ed, mv, n, ctypes.byref(ncand), _stream()),
           "rw_seed_edit_bricks")
    return [bool(ed[i]) for i in range(n)], [float(mv[i]) for i in range(n)]


def _subvols_array(subvols, n):
    if subvols is None:
        return None
    sv = (SubVolume * max(n, 1))()
    for i, (off, (nz, ny, nx), (gz, gy, gx)) in enumerate(subvols):
        sv[i] = SubVolume(int(off), int(nx), int(ny), int(nz), int(gx), int(gy), int(gz))
    return sv


def fill_bricks(coarse_prob, labels, factor, bricks, prob_out, subvols=None, ctx=None):
    """Upsampled coarse probabilities (seeds exact) into the listed bricks of prob_out."""
    ctx = ctx or default_context()
    arr = _bricks_array(bricks)
    _check(lib().rw_fill_bricks(ctx.handle, _ptr(coarse_prob), _dt_code(coarse_prob),
                                _dims(coarse_prob.shape[1:]), int(coarse_prob.shape[0]), int(factor),
                                _ptr(labels), _dims(labels.shape), arr,
                                _subvols_array(subvols, len(bricks)), len(bricks), _ptr(prob_out),
                                _stream()), "rw_fill_bricks")
    return prob_out


# Brick solves refresh their float64 residual when ||r|| fell 100x (whole
# volumes: 10x): measured on 4850 64^3 bricks of a 1024^3 volume, the same CG
# iteration counts with a third fewer refreshes; small, warm-started systems
# keep the float32 recursion close to the true residual over two decades.
BRICK_UPDATE_DELTA = 0.01


def solve_bricks(vol, labels, K, beta, coarse_prob, factor, bricks, prob_out=None, tol=1e-6,
                 precision="mixed", lo=None, hi=None, ctx=None, return_stats=False, subvols=None,
                 workspace=None, **kw):
    """Batched brick solves; returns (prob_out [K][grid] float32, iters [n][R]).

    subvols: None (bricks in `vol`), or per brick (offset, (nz, ny, nx),
    (gz, gy, gx)) of its sub-volume in the flat pool `vol`/`labels`."""
    ctx = ctx or default_context()
    if kw.get("update_delta") is None:
        kw["update_delta"] = BRICK_UPDATE_DELTA
    x0 = kw.get("x0")
    if x0 is not None:
        # initial guess in the layout of prob_out: [K][grid] float32
        if tuple(x0.shape) != (K,) + tuple(vol.shape):
            raise ValueError(f"x0 must be [K][grid] = {(K,) + tuple(vol.shape)}, got "
                             f"{tuple(x0.shape)}")
        kw["x0"] = x0.to(torch.float32).contiguous()
    V = make_volume(vol, lo, hi)
    S = _seeds(labels, K)
    o = options(beta, tol, precision, **kw)
    if prob_out is None:
        prob_out = torch.zeros((K,) + tuple(vol.shape), dtype=torch.float32, device=vol.device)
    arr = _bricks_array(bricks)
    n = len(bricks)
    R = K if o.solve_all_labels else K - 1
    nbytes = lib().rw_bricks_workspace_bytes(arr, n, K, o.precision, o.solve_all_labels)
    ws = workspace if workspace is not None and workspace.numel() >= nbytes else _alloc_ws(
        nbytes, vol.device)
    iters = (ctypes.c_int32 * max(n * R, 1))()
    sv = _subvols_array(subvols, n)
    st = Stats()
    status = lib().rw_solve_bricks(ctx.handle, ctypes.byref(V), ctypes.byref(S), _ptr(coarse_prob),
                                   _dt_code(coarse_prob), _dims(coarse_prob.shape[1:]), int(factor),
                                   arr, sv, n, ctypes.byref(o), _ptr(prob_out), iters, _ptr(ws),
                                   nbytes, ctypes.byref(st), _stream())
    _check(status, "rw_solve_bricks")
    it = [[iters[i * R + r] for r in range(R)] for i in range(n)]
    if return_stats:
        d = st.to_dict()
        d["status"] = status
        return prob_out, it, d
    return prob_out, it


def autotune_bricks(vol, labels, K, beta, coarse_prob, factor, bricks, tol=1e-6,
                    precision="mixed", lo=None, hi=None, ctx=None, subvols=None, **kw):
    """Pick and record the fastest brick tile shape for batches like this one;
    returns (by, rows per lane, zc, xcd order).  Arguments as for solve_bricks."""
    import warnings
    ctx = ctx or default_context()
    if kw.get("update_delta") is None:
        kw["update_delta"] = BRICK_UPDATE_DELTA
    V = make_volume(vol, lo, hi)
    S = _seeds(labels, K)
    o = options(beta, tol, precision, **kw)
    scratch = torch.zeros((K,) + tuple(vol.shape), dtype=torch.float32, device=vol.device)
    arr = _bricks_array(bricks)
    n = len(bricks)
    nbytes = lib().rw_bricks_workspace_bytes(arr, n, K, o.precision, o.solve_all_labels)
    ws = _alloc_ws(nbytes, vol.device)
    sv = _subvols_array(subvols, n)
    best = (ctypes.c_int32 * 4)()
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        _check(lib().rw_autotune_bricks(ctx.handle, ctypes.byref(V), ctypes.byref(S),
                                        _ptr(coarse_prob), _dt_code(coarse_prob),
                                        _dims(coarse_prob.shape[1:]), int(factor), arr, sv, n,
                                        ctypes.byref(o), _ptr(scratch), _ptr(ws), nbytes, best,
                                        _stream()), "rw_autotune_bricks")
    return tuple(best)


def _touches(o, s, roi):
    """Whether the brick (origin o, size s; z, y, x) meets the box roi
    ((z0, z1), (y0, y1), (x0, x1)), half-open."""
    return all(a < hi_ and a + b > lo_ for a, b, (lo_, hi_) in zip(o, s, roi))


def hierarchical_solve(vol, labels, K, beta, levels=2, brick=(64, 64, 64), offset=(0, 0, 0),
                       tol=1e-6, coarse_precision="fp64", brick_precision="mixed", lo=None,
                       hi=None, lo_thr=0.02, hi_thr=0.98, ctx=None, return_info=False,
                       level_dtype=torch.float64, roi=None):
    """Coarse-to-fine random walker: LOD levels, whole coarse solve, brick
    classification, batched solve of the uncertain bricks, upsampled fill of
    the others.  Every step runs in the library; this only sequences calls.

    roi: None (the whole volume) or ((z0, z1), (y0, y1), (x0, x1)), a
    half-open voxel box: lazy evaluation of a requested region (Sec. IV-B's
    evaluation of only what a view needs).  The coarse level is still solved
    whole (it gives every brick its Dirichlet data), but only the bricks that
    meet the box are solved or filled; each brick's solution does not depend
    on which other bricks share its batch, so the box holds exactly what the
    full solve gives there.  Voxels of bricks outside the box are 0."""
    ctx = ctx or default_context()
    V = make_volume(vol, lo, hi)
    g, lab = vol, labels
    glo, ghi = V.norm_lo, V.norm_hi
    for _ in range(levels):
        g, lab = downsample(g, lab, lo=glo, hi=ghi, out_dtype=level_dtype, ctx=ctx)
        glo, ghi = 0.0, 1.0
    coarse, _, cst = solve(g, lab, K, beta, tol=tol, precision=coarse_precision, lo=0.0, hi=1.0,
                           argmax=False, ctx=ctx, return_stats=True)
    f = 2 ** levels
    cands, active = classify_bricks(coarse, labels, f, brick, offset, lo_thr, hi_thr, ctx=ctx)
    want = [roi is None or _touches(o, s, roi) for o, s in cands]
    act = [b for b, a, w in zip(cands, active, want) if a and w]
    ina = [b for b, a, w in zip(cands, active, want) if not a and w]
    alloc = torch.empty if roi is None else torch.zeros
    prob = alloc((K,) + tuple(vol.shape), dtype=torch.float32, device=vol.device)
    if ina:
        fill_bricks(coarse, labels, f, ina, prob, ctx=ctx)
    bst = None
    iters = []
    if act:
        _, iters, bst = solve_bricks(vol, labels, K, beta, coarse, f, act, prob_out=prob, tol=tol,
                                     precision=brick_precision, lo=V.norm_lo, hi=V.norm_hi,
                                     ctx=ctx, return_stats=True,
                                     brick_voxels=int(brick[0]) * brick[1] * brick[2])
    if return_info:
        return prob, dict(coarse=coarse, coarse_stats=cst, bricks=cands, active=active,
                          evaluated=want, brick_iters=iters, brick_stats=bst)
    return prob


def resolve_after_seed_edit(vol, old_labels, new_labels, K, beta, prev_prob, prev_info,
                            levels=2, brick=(64, 64, 64), offset=(0, 0, 0), tol=1e-6,
                            coarse_precision="fp64", brick_precision="mixed", lo=None, hi=None,
                            lo_thr=0.02, hi_thr=0.98, change_tol=1e-4, ctx=None,
                            level_dtype=torch.float64):
    """Warm-started re-solve of a hierarchical solution after seeds changed.

    prev_prob / prev_info: the result of hierarchical_solve(..., return_info=
    True) with old_labels and the same levels, brick grid and thresholds.  The
    coarse level is re-solved from the previous coarse solution; a brick is
    re-solved (from its previous fine solution) or re-filled when it holds an
    edited voxel, when its activity changed, or when the coarse solution
    under it (its coarse footprint and one cell around) moved by more than
    change_tol; every other brick keeps its previous values.  Those differ from
    a full re-solve by at most about change_tol: a brick's solution depends on
    its Dirichlet data through a maximum principle.  Returns (prob, info) with
    info["resolved"] / info["refilled"] the brick indices that were redone."""
    ctx = ctx or default_context()
    V = make_volume(vol, lo, hi)
    g, lab = vol, new_labels
    glo, ghi = V.norm_lo, V.norm_hi
    for _ in range(levels):
        g, lab = downsample(g, lab, lo=glo, hi=ghi, out_dtype=level_dtype, ctx=ctx)
        glo, ghi = 0.0, 1.0
    old_coarse = prev_info["coarse"]
    x0 = old_coarse[1:].to(torch.float64)  # hierarchical_solve solves labels 2..K
    coarse, _, cst = solve(g, lab, K, beta, tol=tol, precision=coarse_precision, lo=0.0, hi=1.0,
                           argmax=False, ctx=ctx, return_stats=True, x0=x0)
    f = 2 ** levels
    cands, active = classify_bricks(coarse, new_labels, f, brick, offset, lo_thr, hi_thr, ctx=ctx)
    if [tuple(map(tuple, b)) for b in cands] != [tuple(map(tuple, b)) for b in
                                                  prev_info["bricks"]]:
        raise ValueError("the brick grid differs from the previous solve's")
    edited, moved = seed_edit_bricks(old_labels, new_labels, old_coarse, coarse, f, brick,
                                     offset, ctx=ctx)
    prob = prev_prob.clone()
    redo = [i for i in range(len(cands))
            if edited[i] or active[i] != prev_info["active"][i] or moved[i] > change_tol]
    solve_ids = [i for i in redo if active[i]]
    fill_ids = [i for i in redo if not active[i]]
    if fill_ids:
        fill_bricks(coarse, new_labels, f, [cands[i] for i in fill_ids], prob, ctx=ctx)
    bst, iters = None, []
    if solve_ids:
        _, iters, bst = solve_bricks(vol, new_labels, K, beta, coarse, f,
                                     [cands[i] for i in solve_ids], prob_out=prob, tol=tol,
                                     precision=brick_precision, lo=V.norm_lo, hi=V.norm_hi,
                                     ctx=ctx, return_stats=True, x0=prev_prob,
                                     brick_voxels=int(brick[0]) * brick[1] * brick[2])
    return prob, dict(coarse=coarse, coarse_stats=cst, bricks=cands, active=active,
                      resolved=solve_ids, refilled=fill_ids, brick_iters=iters, brick_stats=bst,
                      coarse_moved=moved)


# ---------------------------------------------------------------- gradients

def solve_backward(g, labels, K, beta, prob, grad_prob, tol=1e-10, lo=0.0, hi=1.0,
                   solve_all_labels=False, ctx=None, return_stats=False, **kw):
    """Adjoint gradient of a loss of the probabilities prob [K][grid] of a
    float64 solve (dL/dprob = grad_prob [K][grid]): returns (dL/dg on the
    normalised intensities [grid] float64, dL/dbeta as a 0-d float64 device
    tensor).  solve_all_labels must be the forward solve's."""
    ctx = ctx or default_context()
    V = make_volume(g, lo, hi)
    S = _seeds(labels, K)
    o = options(beta, tol, "fp64", solve_all_labels=solve_all_labels, **kw)
    shape = (K,) + tuple(g.shape)
    if tuple(prob.shape) != shape or tuple(grad_prob.shape) != shape:
        raise ValueError(f"prob and grad_prob must be [K][grid] = {shape}")
    prob = prob.to(torch.float64).contiguous()
    grad_prob = grad_prob.to(torch.float64).contiguous()
    grad_g = torch.empty(tuple(g.shape), dtype=torch.float64, device=g.device)
    grad_beta = torch.empty((), dtype=torch.float64, device=g.device)
    nbytes = lib().rw_backward_workspace_bytes(_dims(g.shape))
    ws = _alloc_ws(nbytes, g.device)
    st = Stats()
    status = lib().rw_solve_backward(ctx.handle, ctypes.byref(V), ctypes.byref(S),
                                     ctypes.byref(o), _ptr(prob), _ptr(grad_prob), _ptr(grad_g),
                                     _ptr(grad_beta), _ptr(ws), nbytes, ctypes.byref(st),
                                     _stream())
    _check(status, "rw_solve_backward")
    if return_stats:
        d = st.to_dict()
        d["status"] = status
        return grad_g, grad_beta, d
    return grad_g, grad_beta


class RandomWalkerFn(torch.autograd.Function):
    """Probabilities [K][grid] of a float64 random-walker solve of normalised
    intensities g (GPU, float64) with parameter beta; differentiable in g and
    beta through the library's adjoint solves (rw_solve_backward)."""

    @staticmethod
    def forward(ctx, g, beta, labels, K, tol, solve_all_labels):
        b = float(beta)
        prob, _ = solve(g.contiguous(), labels, K, b, tol=tol, precision="fp64", lo=0.0, hi=1.0,
                        argmax=False, solve_all_labels=solve_all_labels)
        ctx.save_for_backward(g, labels, prob)
        ctx.K, ctx.beta, ctx.tol, ctx.all = K, b, tol, solve_all_labels
        return prob

    @staticmethod
    def backward(ctx, grad_prob):
        g, labels, prob = ctx.saved_tensors
        grad_g, grad_b = solve_backward(g.contiguous(), labels, ctx.K, ctx.beta, prob, grad_prob,
                                        tol=min(ctx.tol, 1e-10), solve_all_labels=ctx.all)
        return grad_g.to(g.dtype), grad_b, None, None, None, None


def random_walker(g, beta, labels, K, tol=1e-10, solve_all_labels=False):
    """Differentiable probabilities [K][grid] (see RandomWalkerFn)."""
    if not torch.is_tensor(beta):
        beta = torch.tensor(float(beta), dtype=torch.float64, device=g.device)
    return RandomWalkerFn.apply(g, beta, labels, K, tol, solve_all_labels)


def argmax(prob, out=None, ctx=None):
    """Label (1..K) of the highest probability per voxel of prob [K][...]
    (float32 or float64, device), lowest label on ties; uint8 [...]."""
    ctx = ctx or default_context()
    prob = prob.contiguous()
    K = int(prob.shape[0])
    if out is None:
        out = torch.empty(tuple(prob.shape[1:]), dtype=torch.uint8, device=prob.device)
    n = prob[0].numel()
    _check(lib().rw_argmax(ctx.handle, _ptr(prob), _dt_code(prob), K, n, _ptr(out), _stream()),
           "rw_argmax")
    return out


def autotune(vol, labels, K, beta, precision="mixed", lo=None, hi=None, ctx=None, **kw):
    """Pick and record the fastest stencil tile shape for this volume; returns (vx, zc, xcd, by)."""
    import warnings
    ctx = ctx or default_context()
    V = make_volume(vol, lo, hi)
    S = _seeds(labels, K)
    o = options(beta, 1e-6, precision, **kw)
    dt = torch.float64 if precision == "fp64" else torch.float32
    prob = torch.empty((K,) + tuple(vol.shape), dtype=dt, device=vol.device)
    nbytes = lib().rw_solve_workspace_bytes(_dims(vol.shape), K, o.precision, o.solve_all_labels)
    ws = _alloc_ws(nbytes, vol.device)
    best = (ctypes.c_int32 * 4)()
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        _check(lib().rw_autotune(ctx.handle, ctypes.byref(V), ctypes.byref(S), ctypes.byref(o),
                                 _ptr(prob), _ptr(ws), nbytes, best, _stream()), "rw_autotune")
    return tuple(best)
