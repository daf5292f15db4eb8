"""ctypes front end of the C oracle (rw_oracle_c.c) — TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg use it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "rw_oracle_c.c")
LIB = os.path.join(_HERE, "liboracle_rw.so")
_lib = None


def build(force=True):
    """Compile the C oracle with gcc (-O2, OpenMP, IEEE arithmetic)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        L.orc_solve_box.argtypes = [P, P, P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                    P, ctypes.c_double, ctypes.c_int, ctypes.c_int, P, P, P]
        L.orc_solve_box.restype = ctypes.c_int
        L.orc_box_weights.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int, P]
        L.orc_box_weights.restype = ctypes.c_int
        L.orc_pcg_fixed_iters.argtypes = [P, P, P, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, P, P]
        L.orc_pcg_fixed_iters.restype = ctypes.c_int
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_last_timing.argtypes = [P, P]
        L.orc_last_timing.restype = None
        L.orc_residual.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int, P,
                                   ctypes.c_int]
        L.orc_residual.restype = ctypes.c_double
        L.orc_adjoint_grad.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double, P, P,
                                       ctypes.c_double, ctypes.c_int, ctypes.c_int, P, P, P, P]
        L.orc_adjoint_grad.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def solve_box(g, labels, label, beta, tol=1e-6, max_iter=20000, box=None, shell=None, x0=None,
              w_eps=0.0, nthreads=0):
    """Jacobi-PCG solve of one label on a box (default: the whole volume).

    g: float64 [nz][ny][nx]; labels: uint8; box = (origin_zyx, size_zyx);
    shell: [sz+2][sy+2][sx+2] Dirichlet values of the non-seed frame voxels;
    x0: [sz][sy][sx].  Returns (x_box, iters, status, rel_true_residual).
    """
    g = np.ascontiguousarray(g, dtype=np.float64)
    labels = np.ascontiguousarray(labels, dtype=np.uint8)
    nz, ny, nx = g.shape
    dims = np.array([nx, ny, nz], dtype=np.int64)
    if box is None:
        box = ((0, 0, 0), (nz, ny, nx))
    (oz, oy, ox), (sz, sy, sx) = box
    b = np.array([ox, oy, oz, sx, sy, sz], dtype=np.int64)
    out = np.empty((sz, sy, sx), dtype=np.float64)
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    sh = None if shell is None else np.ascontiguousarray(shell, dtype=np.float64)
    x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    st = lib().orc_solve_box(_p(g), _p(labels), _p(dims), _p(b),
                             None if sh is None else _p(sh), float(beta), float(w_eps), int(label),
                             None if x0a is None else _p(x0a), float(tol), int(max_iter),
                             int(nthreads), _p(out), ctypes.byref(it), ctypes.byref(rel))
    return out, it.value, st, rel.value


def random_walker(g, labels, K, beta, tol=1e-6, max_iter=20000, solve_labels=None, nthreads=0,
                  return_info=False):
    """All labels (default) solved independently on the whole volume."""
    solve_labels = list(range(1, K + 1)) if solve_labels is None else list(solve_labels)
    out = np.empty((len(solve_labels),) + tuple(np.shape(g)))
    info = []
    for k, s in enumerate(solve_labels):
        x, it, st, rel = solve_box(g, labels, s, beta, tol, max_iter, nthreads=nthreads)
        out[k] = x
        info.append(dict(label=s, iters=it, status=st, rel_residual=rel))
    return (out, info) if return_info else out


def box_weights(g, beta, box=None, w_eps=0.0, nthreads=0):
    g = np.ascontiguousarray(g, dtype=np.float64)
    nz, ny, nx = g.shape
    dims = np.array([nx, ny, nz], dtype=np.int64)
    if box is None:
        box = ((0, 0, 0), (nz, ny, nx))
    (oz, oy, ox), (sz, sy, sx) = box
    b = np.array([ox, oy, oz, sx, sy, sz], dtype=np.int64)
    w6 = np.empty((6, sz, sy, sx))
    lib().orc_box_weights(_p(g), _p(dims), _p(b), float(beta), float(w_eps), int(nthreads), _p(w6))
    return w6


def pcg_fixed_iters(g, labels, label, beta, n_iter, nthreads=0):
    """Run exactly n_iter PCG iterations on the whole volume (timing samples)."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    labels = np.ascontiguousarray(labels, dtype=np.uint8)
    nz, ny, nx = g.shape
    dims = np.array([nx, ny, nz], dtype=np.int64)
    out = np.empty(g.shape)
    it = ctypes.c_int(0)
    st = lib().orc_pcg_fixed_iters(_p(g), _p(labels), _p(dims), float(beta), int(label),
                                   int(n_iter), int(nthreads), _p(out), ctypes.byref(it))
    return out, it.value, st


def max_threads():
    return lib().orc_max_threads()


def last_timing():
    """(set-up seconds, CG-loop seconds) of the last solve."""
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().orc_last_timing(ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def residual(g, labels, label, beta, x, w_eps=0.0, nthreads=0):
    """Float64 relative residual ||b - A x|| / ||b|| of a full-grid x of one label."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    labels = np.ascontiguousarray(labels, dtype=np.uint8)
    x = np.ascontiguousarray(x, dtype=np.float64)
    nz, ny, nx = g.shape
    dims = np.array([nx, ny, nz], dtype=np.int64)
    return float(lib().orc_residual(_p(g), _p(labels), _p(dims), float(beta), float(w_eps),
                                    int(label), _p(x), int(nthreads)))


def adjoint_gradient(g, labels, beta, x_full, dLdx, tol=1e-12, max_iter=200000, w_eps=0.0,
                     nthreads=0):
    """dL/dbeta and dL/dg of a loss of one label's whole-volume solution x_full
    (seeds exact) with dL/dx = dLdx: the adjoint system L_U lam = dL/dx_U solved
    by the oracle's Jacobi-PCG to `tol`, then the per-edge sums.  Returns
    (dL/dbeta, dL/dg [nz][ny][nx], lam, iterations, status)."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    labels = np.ascontiguousarray(labels, dtype=np.uint8)
    x_full = np.ascontiguousarray(x_full, dtype=np.float64)
    dLdx = np.ascontiguousarray(dLdx, dtype=np.float64)
    nz, ny, nx = g.shape
    dims = np.array([nx, ny, nz], dtype=np.int64)
    lam = np.empty(g.shape)
    dg = np.empty(g.shape)
    db = ctypes.c_double(0.0)
    it = ctypes.c_int(0)
    st = lib().orc_adjoint_grad(_p(g), _p(labels), _p(dims), float(beta), float(w_eps),
                                _p(x_full), _p(dLdx), float(tol), int(max_iter), int(nthreads),
                                _p(lam), _p(dg), ctypes.byref(db), ctypes.byref(it))
    return db.value, dg, lam, it.value, st
