"""ctypes front-end of the C oracle (md_oracle.c).  Test infrastructure only.

Arrays are numpy, C-contiguous: positions/velocities/forces [n, 2] float64,
image counts [n, 2] int64, counts [50] int64, dense fields [49, lx, lx] int32.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import lattice

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle_md.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


class _CG(C.Structure):
    _fields_ = [
        ("lx", C.c_int32),
        ("s_cg", C.c_int32),
        ("ux", C.c_double),
        ("uy", C.c_double),
        ("k0", C.c_int64),
        ("vtab", C.c_void_p),
        ("counts", C.c_void_p),
        ("cell_acc", C.c_void_p),
        ("moments", C.c_void_p),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIBPATH)
    lib.orc_forces_brute.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_double, C.c_int32,
                                     _dp, _dp, C.POINTER(C.c_double)]
    lib.orc_forces_cells.argtypes = lib.orc_forces_brute.argtypes
    lib.orc_energy.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int32,
                               _dp, _dp, _dp]
    lib.orc_coarse_grain.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, _i32p, C.c_int64,
                                     _dp, C.c_void_p, C.c_int64, _dp, C.c_void_p, C.c_int64,
                                     _i64p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.orc_coarse_grain_shift.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double,
                                           C.c_double, _i32p, C.c_int64, _dp, C.c_void_p, _dp, C.c_void_p,
                                           _i64p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.orc_coarse_grain_literal.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, _i32p,
                                             C.c_int64, _dp, C.c_int64, _dp, C.c_int64, _i64p,
                                             C.c_void_p]
    lib.orc_neq_mdlg.argtypes = [C.c_int32, C.c_double, _i32p, C.c_int32, _i64p, C.c_int32, C.c_int64, _dp, _i64p,
                                 _i32p, _i64p, C.c_void_p]
    lib.orc_neq_mdlg.restype = C.c_int
    lib.orc_displacement_hist.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_int32, _dp, C.c_void_p, _dp,
                                          C.c_void_p, _i64p]
    lib.orc_md_run.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32,
                               C.c_int32, C.c_int64, _dp, _dp, _i64p, C.POINTER(_CG), C.c_void_p,
                               C.c_int64]
    lib.orc_md_run.restype = C.c_int64
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def forces(pos, L, rc=2.5, eps=1.0, shift=True, method="cells"):
    """LJ forces [n, 2] and the potential energy of a configuration."""
    lib = _load()
    pos = _f64(pos)
    n = pos.shape[0]
    f = np.zeros((n, 2))
    pe = C.c_double(0.0)
    fn = lib.orc_forces_cells if method == "cells" else lib.orc_forces_brute
    fn(n, L, rc, eps, 1 if shift else 0, pos, f, C.byref(pe))
    return f, pe.value


def energy(pos, vel, L, rc=2.5, eps=1.0, shift=True, cells=True):
    """(KE, PE, Px, Py) with compensated sums."""
    lib = _load()
    pos, vel = _f64(pos), _f64(vel)
    out = np.zeros(4)
    lib.orc_energy(pos.shape[0], L, rc, eps, 1 if shift else 0, 1 if cells else 0, pos, vel, out)
    return out


class CGAccum:
    """Accumulators of a coarse-graining run: counts [50], optional cell_acc, moments [5]."""

    def __init__(self, lx, cell_acc=False):
        self.lx = lx
        self.counts = np.zeros(50, dtype=np.int64)
        self.cell_acc = np.zeros((49, lx, lx), dtype=np.int32) if cell_acc else None
        self.moments = np.zeros(5)
        self.events = 0


def md_run(pos, vel, img, L, nsteps, dt=1e-4, rc=2.5, eps=1.0, shift=True, cells=True,
           cg: CGAccum | None = None, s_cg=0, u=(0.0, 0.0), k0=0, energy_every=0):
    """Velocity-Verlet run of nsteps steps.  pos/vel/img are updated in place
    (copies are made if they are not contiguous of the right dtype and then
    returned).  Returns (pos, vel, img, energy_trace or None)."""
    lib = _load()
    pos, vel, img = _f64(pos), _f64(vel), _i64(img)
    n = pos.shape[0]
    vtab = lattice.d2q49()
    cgs = None
    if cg is not None and s_cg > 0:
        cgs = _CG(lx=cg.lx, s_cg=s_cg, ux=u[0], uy=u[1], k0=k0, vtab=_ptr(vtab),
                  counts=_ptr(cg.counts), cell_acc=_ptr(cg.cell_acc), moments=_ptr(cg.moments))
    etrace = None
    if energy_every > 0:
        etrace = np.zeros((nsteps // energy_every + 1, 4))
    ev = lib.orc_md_run(n, L, dt, rc, eps, 1 if shift else 0, 1 if cells else 0, nsteps, pos, vel, img,
                        C.byref(cgs) if cgs is not None else None, _ptr(etrace), energy_every)
    if cg is not None:
        cg.events += int(ev)
    return pos, vel, img, etrace


def coarse_grain(lx, L, pos_prev, pos_cur, img_prev=None, img_cur=None, k_prev=0, k_cur=1,
                 u=(0.0, 0.0), counts=None, cell_acc=None, moments=None, dense=False):
    """One binned coarse-graining event.  Returns (counts, n_event or None, moments)."""
    lib = _load()
    pos_prev, pos_cur = _f64(pos_prev), _f64(pos_cur)
    n = pos_prev.shape[0]
    vtab = lattice.d2q49()
    counts = np.zeros(50, dtype=np.int64) if counts is None else counts
    moments = np.zeros(5) if moments is None else moments
    n_event = np.zeros((49, lx, lx), dtype=np.int32) if dense else None
    ip = None if img_prev is None else _i64(img_prev)
    ic = None if img_cur is None else _i64(img_cur)
    lib.orc_coarse_grain(lx, L, u[0], u[1], vtab, n, pos_prev, _ptr(ip), k_prev, pos_cur, _ptr(ic), k_cur,
                         counts, _ptr(n_event), _ptr(cell_acc), _ptr(moments))
    return counts, n_event, moments


def coarse_grain_shift(lx, L, pos_prev, pos_cur, img_prev, img_cur, shift_prev, shift_cur, counts=None,
                       moments=None):
    """One binned event on a lattice translated by shift_prev / shift_cur (lengths, [2] each).
    Returns (counts, moments)."""
    lib = _load()
    pos_prev, pos_cur = _f64(pos_prev), _f64(pos_cur)
    n = pos_prev.shape[0]
    vtab = lattice.d2q49()
    counts = np.zeros(50, dtype=np.int64) if counts is None else counts
    moments = np.zeros(5) if moments is None else moments
    ip = None if img_prev is None else _i64(img_prev)
    ic = None if img_cur is None else _i64(img_cur)
    lib.orc_coarse_grain_shift(lx, L, float(shift_prev[0]), float(shift_prev[1]), float(shift_cur[0]),
                               float(shift_cur[1]), vtab, n, pos_prev, _ptr(ip), pos_cur, _ptr(ic), counts, None,
                               None, _ptr(moments))
    return counts, moments


def coarse_grain_literal(lx, L, pos_prev, pos_cur, k_prev=0, k_cur=1, u=(0.0, 0.0)):
    """Literal Eq.(n_i) over the periodic lattice.  Returns (counts [50], n_event [49, lx, lx])."""
    lib = _load()
    pos_prev, pos_cur = _f64(pos_prev), _f64(pos_cur)
    vtab = lattice.d2q49()
    counts = np.zeros(50, dtype=np.int64)
    n_event = np.zeros((49, lx, lx), dtype=np.int32)
    lib.orc_coarse_grain_literal(lx, L, u[0], u[1], vtab, pos_prev.shape[0], pos_prev, k_prev, pos_cur,
                                 k_cur, counts, _ptr(n_event))
    return counts, n_event


def displacement_hist(L, h, n_bin, pos_prev, pos_cur, img_prev=None, img_cur=None, hist=None):
    """Per-axis histogram of the box-frame displacements of one snapshot pair
    (bins of width h, see orc_displacement_hist).  Returns hist [2, n_bin + 2] int64."""
    lib = _load()
    pos_prev, pos_cur = _f64(pos_prev), _f64(pos_cur)
    hist = np.zeros((2, n_bin + 2), dtype=np.int64) if hist is None else hist
    ip = None if img_prev is None else _i64(img_prev)
    ic = None if img_cur is None else _i64(img_cur)
    lib.orc_displacement_hist(pos_prev.shape[0], float(L), float(h), int(n_bin), pos_prev, _ptr(ip), pos_cur,
                              _ptr(ic), hist)
    return hist


def displacement_hist_series(offsets, box_l, pos, img, lags, h, n_bin):
    """Displacement histograms of a stacked trajectory pos [P, n_tot, 2], img [P, n_tot, 2]:
    for replica r (particles offsets[r] .. offsets[r+1]-1, box side box_l[r]) and lag
    lags[s] (bin width h[s]), every snapshot pair (p - lag, p).
    Returns [n_rep, n_lag, 2, n_bin + 2] int64."""
    offsets = [int(o) for o in offsets]
    n_rep, n_snap = len(offsets) - 1, pos.shape[0]
    out = np.zeros((n_rep, len(lags), 2, n_bin + 2), dtype=np.int64)
    for r in range(n_rep):
        a, b = offsets[r], offsets[r + 1]
        if b == a:
            continue
        for s, lag in enumerate(lags):
            for p in range(lag, n_snap):
                displacement_hist(box_l[r], h[s], n_bin, pos[p - lag, a:b], pos[p, a:b], img[p - lag, a:b],
                                  img[p, a:b], hist=out[r, s])
    return out


def neq_mdlg(lx, L, offsets, pos, img, xi=True):
    """Ensemble sums over replica trajectories pos/img [P, n_tot, 2] (see orc_neq_mdlg).
    Returns (f_sum [P-1, 49, lx, lx] int32, ovf [P-1] int64, xi_sum [P-2, 49, lx, lx] int32 or None)."""
    lib = _load()
    pos = _f64(pos)
    img = _i64(img)
    P, n_tot = pos.shape[0], pos.shape[1]
    off = _i64(offsets)
    f_sum = np.zeros((P - 1, 49, lx, lx), dtype=np.int32)
    ovf = np.zeros(P - 1, dtype=np.int64)
    xi_sum = np.zeros((max(P - 2, 0), 49, lx, lx), dtype=np.int32) if xi else None
    rc = lib.orc_neq_mdlg(int(lx), float(L), lattice.d2q49(), len(off) - 1, off, P, n_tot, pos, img, f_sum, ovf,
                          _ptr(xi_sum) if xi and P > 2 else None)
    if rc != 0:
        raise MemoryError("orc_neq_mdlg")
    return f_sum, ovf, xi_sum


def vacf_sums(offsets, vel, lags):
    """Velocity autocorrelation sums of stacked velocity snapshots vel [P, n_tot, 2]:
    out[r, s] = sum over particles j of replica r and origins p = 0 .. P-1-lag of
    v_j(p) . v_j(p + lag), lag = lags[s], summed in FP64 (numpy pairwise order).
    Returns [n_rep, n_lag] float64."""
    vel = _f64(vel)
    P = vel.shape[0]
    offsets = [int(o) for o in offsets]
    out = np.zeros((len(offsets) - 1, len(lags)))
    for r in range(len(offsets) - 1):
        a, b = offsets[r], offsets[r + 1]
        for s, lag in enumerate(lags):
            if b > a:
                out[r, s] = float(np.sum(vel[:P - lag, a:b] * vel[lag:, a:b]))
    return out
