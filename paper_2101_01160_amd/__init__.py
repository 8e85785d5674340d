"""MI355X hot path of the molecular dynamics lattice gas (MDLG) method.

Thin Python binding of libmdlg.so (C ABI: include/mdlg.h).  Functions carry
the C names and only marshal arguments: torch tensors supply device memory
and the current HIP stream; every step of the computation runs in the
library's HIP kernels (or, for the closed forms, in its host FP64 code).

Quick use::

    sys = LJSystem(pos0, vel0, box_l=L)              # torch float64 [n, 2] on cuda
    acc = sys.attach_cg(lx=1024, s_cg=50)             # fused coarse-graining
    sys.step(20_000)
    g, ovf = mdlg_feq_measured(acc.counts.cpu().numpy(), n, acc.events)
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import _abi
from ._abi import Info, LJParams, Lattice, MDLGError

__all__ = [
    "MDLGError", "LJParams", "Lattice", "LJSystem", "CGAccumulators",
    "lj_params", "lj_md_init", "lj_md_init_batch", "lj_md_cg_attach", "lj_md_cg_detach", "lj_md_step", "lj_md_step_timed",
    "lj_md_get_state", "lj_md_forces", "lj_md_energy", "lj_md_check", "lj_md_info", "lj_md_save", "lj_md_load",
    "lj_md_destroy",
    "lj_md_autotune",
    "mdlg_coarse_grain", "mdlg_coarse_grain_series", "mdlg_feq_measured", "NOALLOC_MAX_N", "mdlg_moments", "mdlg_lambda_from_moments",
    "mdlg_feq_gauss", "mdlg_feq_wsg", "mdlg_velocity_table", "mdlg_version",
    "mdlg_neq_mdlg", "mdlg_vacf", "mdlg_lambda_vacf", "mdlg_displacement_hist", "mdlg_pdf_bins", "mdlg_pdf_measured", "mdlg_kl_divergence",
    "mdlg_mlp_create", "mdlg_mlp_params", "mdlg_mlp_forward", "mdlg_mlp_gradient", "mdlg_mlp_train_step",
    "mdlg_feq_surrogate", "mdlg_mlp_destroy", "SurrogateMLP", "MLP_NPARAMS",
    "mdlg_moment_table_create", "mdlg_moment_table_eval", "mdlg_moment_table_info", "mdlg_moment_table_destroy",
    "mdlg_feq_surrogate_table", "MomentTable",
]

MLP_NPARAMS = _abi.MLP_NPARAMS
NOALLOC_MAX_N = _abi.NOALLOC_MAX_N


def _torch():
    import torch
    return torch


def _stream(stream):
    if stream is None:
        return C.c_void_p(_torch().cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _check(t, dtype, shape, name):
    """dtype, shape and layout of a tensor argument (None passes)."""
    if t is None:
        return
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor on the GPU")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _dev(t, dtype, shape=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (None passes NULL)."""
    if t is None:
        return None
    _check(t, dtype, shape, name)
    if not t.is_cuda:
        raise ValueError(f"{name} must be a torch tensor on the GPU")
    return C.c_void_p(t.data_ptr())


def _devs(*specs):
    """Device pointers of several (tensor, dtype, shape, name) arguments; every
    dtype and shape is checked before any device test, so that a wrongly sized
    buffer is refused first and nothing reaches the library."""
    for t, dtype, shape, name in specs:
        _check(t, dtype, shape, name)
    return [_dev(*sp) for sp in specs]


def _host(a, dtype, n):
    a = np.ascontiguousarray(a, dtype=dtype)
    if a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def mdlg_version() -> str:
    return _abi.lib().mdlg_version().decode()


def mdlg_velocity_table() -> np.ndarray:
    out = np.zeros((49, 2), np.int32)
    _abi.check(_abi.lib().mdlg_velocity_table(out.ctypes.data_as(C.c_void_p)))
    return out


# ------------------------------------------------------------------ MD ---

def lj_params(n, box_l, dt=1e-4, rc=2.5, eps=1.0, energy_shift=True, force_bits=64, skin=0.0,
              rebuild_every=0, block_size=0, step_kernel=0, gather_batch=0, fuse_steps=0) -> LJParams:
    return LJParams(n=int(n), box_l=float(box_l), dt=float(dt), rc=float(rc), eps=float(eps),
                    energy_shift=1 if energy_shift else 0, force_bits=int(force_bits), skin=float(skin),
                    rebuild_every=int(rebuild_every), block_size=int(block_size), step_kernel=int(step_kernel),
                    gather_batch=int(gather_batch), fuse_steps=int(fuse_steps))


def lj_md_init(params: LJParams, pos0, vel0, stream=None) -> C.c_void_p:
    torch = _torch()
    n = params.n
    h = C.c_void_p()
    _abi.check(_abi.lib().lj_md_init(C.byref(h), C.byref(params), _dev(pos0, torch.float64, (n, 2), "pos0"),
                                     _dev(vel0, torch.float64, (n, 2), "vel0"), _stream(stream)))
    return h


def lj_md_init_batch(params, pos0, vel0, stream=None) -> C.c_void_p:
    torch = _torch()
    arr = (LJParams * len(params))(*params)
    n = sum(p.n for p in params)
    h = C.c_void_p()
    _abi.check(_abi.lib().lj_md_init_batch(C.byref(h), len(params), arr, _dev(pos0, torch.float64, (n, 2), "pos0"),
                                           _dev(vel0, torch.float64, (n, 2), "vel0"), _stream(stream)))
    return h


def _sizes(h):
    """(replicas, particles) of a handle: the extents every per-handle buffer is checked against."""
    info = lj_md_info(h)
    return int(info["n_rep"]), int(info["n_total"])


def lj_md_cg_attach(h, s_cg, lattices, counts, moments, cell_acc=None, stream=None):
    """counts: int64 [n_rep, 50], moments: float64 [n_rep, 5], cell_acc: int32
    [sum over replicas of 49 lx^2] or None (all on the GPU, accumulated into)."""
    torch = _torch()
    n_rep, _ = _sizes(h)
    if len(lattices) != n_rep:
        raise ValueError(f"expected {n_rep} lattices, got {len(lattices)}")
    lats = (Lattice * len(lattices))(*lattices)
    n_cells = sum(49 * int(l.lx) * int(l.lx) for l in lattices)
    ptrs = _devs((counts, torch.int64, (n_rep, 50), "counts"), (moments, torch.float64, (n_rep, 5), "moments"),
                 (cell_acc, torch.int32, (n_cells,), "cell_acc"))
    _abi.check(_abi.lib().lj_md_cg_attach(h, int(s_cg), lats, *ptrs, _stream(stream)))


def lj_md_cg_detach(h):
    _abi.check(_abi.lib().lj_md_cg_detach(h))


def lj_md_step(h, nsteps, stream=None):
    _abi.check(_abi.lib().lj_md_step(h, int(nsteps), _stream(stream)))


def lj_md_step_timed(h, nunits, stream=None, sample_every=1):
    """Advance nunits cell-list intervals, timing every sample_every-th one as split graphs.  Returns
    (avg ms [3], counts [3]) for [ordinary step kernel, coarse-graining step with the launches after it,
    cell-list rebuild]."""
    ms = np.zeros(3)
    cnt = np.zeros(3, np.int32)
    _abi.check(_abi.lib().lj_md_step_timed(h, int(nunits), int(sample_every), ms.ctypes.data_as(C.c_void_p),
                                           cnt.ctypes.data_as(C.c_void_p), _stream(stream)))
    return ms, cnt


def lj_md_get_state(h, pos=None, vel=None, img=None, stream=None):
    """pos, vel: float64 [n_total, 2], img: int32 [n_total, 2] on the GPU, in caller order (each may be None)."""
    torch = _torch()
    _, n = _sizes(h)
    ptrs = _devs((pos, torch.float64, (n, 2), "pos"), (vel, torch.float64, (n, 2), "vel"),
                 (img, torch.int32, (n, 2), "img"))
    _abi.check(_abi.lib().lj_md_get_state(h, *ptrs, _stream(stream)))


def lj_md_save(h, path, stream=None):
    _abi.check(_abi.lib().lj_md_save(h, os.fsencode(path), _stream(stream)))


def lj_md_load(path, stream=None) -> C.c_void_p:
    h = C.c_void_p()
    _abi.check(_abi.lib().lj_md_load(C.byref(h), os.fsencode(path), _stream(stream)))
    return h


def lj_md_forces(h, force, stream=None):
    """force: float64 [n_total, 2] on the GPU, caller order."""
    _, n = _sizes(h)
    _abi.check(_abi.lib().lj_md_forces(h, _dev(force, _torch().float64, (n, 2), "force"), _stream(stream)))


def lj_md_energy(h, stream=None) -> np.ndarray:
    """(KE, PE, Px, Py) per replica, [n_rep, 4] (synchronises)."""
    n_rep, _ = _sizes(h)
    out = np.zeros((n_rep, 4))
    _abi.check(_abi.lib().lj_md_energy(h, out.ctypes.data_as(C.c_void_p), _stream(stream)))
    return out


def lj_md_check(h, stream=None):
    _abi.check(_abi.lib().lj_md_check(h, _stream(stream)))


def lj_md_info(h) -> dict:
    info = Info()
    _abi.check(_abi.lib().lj_md_info(h, C.byref(info)))
    return {k: getattr(info, k) for k, _ in Info._fields_}


def lj_md_destroy(h):
    if h:
        _abi.lib().lj_md_destroy(h)


def lj_md_autotune(params, pos0, vel0, s_cg=0, lattices=None, use_cache=True, stream=None):
    """Tuned copies of `params` (list of LJParams) and the best time per MD step in us
    (-1 when taken from the cache)."""
    torch = _torch()
    n = sum(p.n for p in params)
    arr_in = (LJParams * len(params))(*params)
    arr_out = (LJParams * len(params))()
    lats = None if lattices is None else (Lattice * len(lattices))(*lattices)
    us = C.c_double()
    _abi.check(_abi.lib().lj_md_autotune(len(params), arr_in, _dev(pos0, torch.float64, (n, 2), "pos0"),
                                         _dev(vel0, torch.float64, (n, 2), "vel0"), int(s_cg), lats,
                                         0 if use_cache else 1, arr_out, C.byref(us), _stream(stream)))
    return list(arr_out), us.value


# ------------------------------------------------------- coarse-graining ---

def mdlg_coarse_grain(lx, box_l, pos_prev, pos_cur, counts, moments=None, img_prev=None, img_cur=None,
                      k_prev=0, k_cur=1, u=(0.0, 0.0), n_event=None, cell_acc=None, stream=None, noalloc=False):
    """One coarse-graining event between two snapshots (see include/mdlg.h).
    noalloc=True calls mdlg_coarse_grain_noalloc (no device allocation; at
    most NOALLOC_MAX_N particles)."""
    torch = _torch()
    n = pos_prev.shape[0]
    lat = Lattice(lx=int(lx), reserved=0, u=(C.c_double * 2)(float(u[0]), float(u[1])))
    fn = _abi.lib().mdlg_coarse_grain_noalloc if noalloc else _abi.lib().mdlg_coarse_grain
    _abi.check(fn(
        C.byref(lat), float(box_l), int(n),
        _dev(pos_prev, torch.float64, (n, 2), "pos_prev"), _dev(img_prev, torch.int32, (n, 2), "img_prev"),
        int(k_prev),
        _dev(pos_cur, torch.float64, (n, 2), "pos_cur"), _dev(img_cur, torch.int32, (n, 2), "img_cur"), int(k_cur),
        _dev(counts, torch.int64, (50,), "counts"), _dev(moments, torch.float64, (5,), "moments"),
        _dev(n_event, torch.int32, (49, lx, lx), "n_event"), _dev(cell_acc, torch.int32, (49, lx, lx), "cell_acc"),
        _stream(stream)))


def mdlg_coarse_grain_series(offsets, box_l, lx, pos, img, lags, u, counts, moments=None, lattice_offset=None,
                             stream=None):
    """pos: torch float64 [P, n_tot, 2], img: torch int32 [P, n_tot, 2] on the GPU;
    counts: torch int64 [n_rep, n_lag, n_u, 50]; moments: torch float64 [n_rep, n_lag, 5];
    lattice_offset: host [P, 2] lattice origin (cells) of the pairs starting at each snapshot."""
    torch = _torch()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    n_rep = off.size - 1
    box = _host(box_l, np.float64, n_rep)
    lxs = _host(lx, np.int32, n_rep)
    lg = np.ascontiguousarray(lags, dtype=np.int32).ravel()
    uu = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 2)
    P, n_tot = int(pos.shape[0]), int(pos.shape[1])
    lo = None if lattice_offset is None else _host(lattice_offset, np.float64, 2 * P)
    if n_tot != int(off[-1]):
        raise ValueError("pos holds a different particle count than offsets")
    _abi.check(_abi.lib().mdlg_coarse_grain_series(
        int(n_rep), off.ctypes.data_as(C.c_void_p), box.ctypes.data_as(C.c_void_p),
        lxs.ctypes.data_as(C.c_void_p), P, _dev(pos, torch.float64, (P, n_tot, 2), "pos"),
        _dev(img, torch.int32, (P, n_tot, 2), "img"), int(lg.size), lg.ctypes.data_as(C.c_void_p),
        int(uu.shape[0]), uu.ctypes.data_as(C.c_void_p), None if lo is None else lo.ctypes.data_as(C.c_void_p),
        _dev(counts, torch.int64, (n_rep, lg.size, uu.shape[0], 50), "counts"),
        _dev(moments, torch.float64, (n_rep, lg.size, 5), "moments"), _stream(stream)))


def mdlg_vacf(offsets, vel, lags, c_sum, stream=None):
    """vel: torch float64 [P, n_tot, 2] on the GPU; c_sum: torch float64 [n_rep, n_lag] on the GPU (added to)."""
    torch = _torch()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    n_rep = off.size - 1
    lg = np.ascontiguousarray(lags, dtype=np.int32).ravel()
    P, n_tot = int(vel.shape[0]), int(vel.shape[1])
    if n_tot != int(off[-1]):
        raise ValueError("vel holds a different particle count than offsets")
    _abi.check(_abi.lib().mdlg_vacf(int(n_rep), off.ctypes.data_as(C.c_void_p), P,
                                    _dev(vel, torch.float64, (P, n_tot, 2), "vel"), int(lg.size),
                                    lg.ctypes.data_as(C.c_void_p), _dev(c_sum, torch.float64, (n_rep, lg.size), "c_sum"),
                                    _stream(stream)))


def mdlg_lambda_vacf(t, c, dt_cg, cut=0.01):
    """(tau, lambda) from sampled C(t)."""
    tt = np.ascontiguousarray(t, dtype=np.float64).ravel()
    cc = _host(c, np.float64, tt.size)
    tau, lam = C.c_double(), C.c_double()
    _abi.check(_abi.lib().mdlg_lambda_vacf(int(tt.size), tt.ctypes.data_as(C.c_void_p), cc.ctypes.data_as(C.c_void_p),
                                           float(dt_cg), float(cut), C.byref(tau), C.byref(lam)))
    return tau.value, lam.value


def mdlg_neq_mdlg(box_l, lx, pos, img, f_sum, overflow, xi_sum=None, stream=None):
    """pos: torch float64 [P, n_total, 2], img: torch int32 [P, n_total, 2] on the GPU (an ensemble of
    replicas of one system, snapshots one coarse step apart); outputs (overwritten): f_sum int32
    [P-1, 49, lx, lx], overflow int64 [P-1], xi_sum int32 [P-2, 49, lx, lx] or None."""
    torch = _torch()
    P, n = int(pos.shape[0]), int(pos.shape[1])
    lx = int(lx)
    _abi.check(_abi.lib().mdlg_neq_mdlg(
        n, float(box_l), lx, P, _dev(pos, torch.float64, (P, n, 2), "pos"), _dev(img, torch.int32, (P, n, 2), "img"),
        _dev(f_sum, torch.int32, (P - 1, 49, lx, lx), "f_sum"), _dev(overflow, torch.int64, (P - 1,), "overflow"),
        _dev(xi_sum, torch.int32, (max(P - 2, 0), 49, lx, lx), "xi_sum"), _stream(stream)))


def mdlg_displacement_hist(offsets, box_l, pos, img, lags, bin_width, n_bin, hist, stream=None):
    """pos: torch float64 [P, n_tot, 2], img: torch int32 [P, n_tot, 2] on the GPU;
    hist: torch int64 [n_rep, n_lag, 2, n_bin + 2] on the GPU (added to)."""
    torch = _torch()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    n_rep = off.size - 1
    box = _host(box_l, np.float64, n_rep)
    lg = np.ascontiguousarray(lags, dtype=np.int32).ravel()
    bw = _host(bin_width, np.float64, lg.size)
    P, n_tot = int(pos.shape[0]), int(pos.shape[1])
    if n_tot != int(off[-1]):
        raise ValueError("pos holds a different particle count than offsets")
    _abi.check(_abi.lib().mdlg_displacement_hist(
        int(n_rep), off.ctypes.data_as(C.c_void_p), box.ctypes.data_as(C.c_void_p), P,
        _dev(pos, torch.float64, (P, n_tot, 2), "pos"), _dev(img, torch.int32, (P, n_tot, 2), "img"),
        int(lg.size), lg.ctypes.data_as(C.c_void_p), bw.ctypes.data_as(C.c_void_p), int(n_bin),
        _dev(hist, torch.int64, (n_rep, lg.size, 2, int(n_bin) + 2), "hist"), _stream(stream)))


def mdlg_pdf_bins(msd, lam, mean, h, n_bin):
    """(P^G, P^WSG) bin probabilities, float64 [n_bin + 2] each (tails last)."""
    pg = np.zeros(int(n_bin) + 2)
    pw = np.zeros(int(n_bin) + 2)
    _abi.check(_abi.lib().mdlg_pdf_bins(float(msd), float(lam), float(mean), float(h), int(n_bin),
                                        pg.ctypes.data_as(C.c_void_p), pw.ctypes.data_as(C.c_void_p)))
    return pg, pw


def mdlg_pdf_measured(hist):
    """P^MD: host histograms [..., n] pooled over the leading axes and normalised."""
    h = np.ascontiguousarray(hist, dtype=np.int64)
    n = int(h.shape[-1])
    h = h.reshape(-1, n)
    p = np.zeros(n)
    _abi.check(_abi.lib().mdlg_pdf_measured(h.ctypes.data_as(C.c_void_p), int(h.shape[0]), n,
                                            p.ctypes.data_as(C.c_void_p)))
    return p


def mdlg_kl_divergence(r, q):
    """(K(X_i) [n], D_KL(R || Q))."""
    rr = np.ascontiguousarray(r, dtype=np.float64).ravel()
    qq = _host(q, np.float64, rr.size)
    k = np.zeros(rr.size)
    d = C.c_double()
    _abi.check(_abi.lib().mdlg_kl_divergence(rr.ctypes.data_as(C.c_void_p), qq.ctypes.data_as(C.c_void_p),
                                             int(rr.size), k.ctypes.data_as(C.c_void_p), C.byref(d)))
    return k, d.value


# ------------------------------------------------------------ equilibria ---

def mdlg_feq_measured(counts, n_particles, n_events, symmetrize=False):
    c = _host(counts, np.int64, 50)
    g = np.zeros(49)
    ovf = C.c_double()
    _abi.check(_abi.lib().mdlg_feq_measured(c.ctypes.data_as(C.c_void_p), int(n_particles), int(n_events),
                                            1 if symmetrize else 0, g.ctypes.data_as(C.c_void_p), C.byref(ovf)))
    return g, ovf.value


def mdlg_moments(moments, dx):
    m = _host(moments, np.float64, 5)
    mu2, mu4, a2 = C.c_double(), C.c_double(), C.c_double()
    _abi.check(_abi.lib().mdlg_moments(m.ctypes.data_as(C.c_void_p), float(dx), C.byref(mu2), C.byref(mu4),
                                       C.byref(a2)))
    return mu2.value, mu4.value, a2.value


def mdlg_lambda_from_moments(mu2, mu4, branch=2):
    lam, r = C.c_double(), C.c_double()
    _abi.check(_abi.lib().mdlg_lambda_from_moments(float(mu2), float(mu4), int(branch), C.byref(lam), C.byref(r)))
    return lam.value, r.value


def mdlg_feq_gauss(a2, u=(0.0, 0.0)):
    uu = _host(u, np.float64, 2)
    g = np.zeros(49)
    _abi.check(_abi.lib().mdlg_feq_gauss(float(a2), uu.ctypes.data_as(C.c_void_p), g.ctypes.data_as(C.c_void_p)))
    return g


def mdlg_feq_wsg(a2, lam, u=(0.0, 0.0)):
    uu = _host(u, np.float64, 2)
    g = np.zeros(49)
    _abi.check(_abi.lib().mdlg_feq_wsg(float(a2), float(lam), uu.ctypes.data_as(C.c_void_p),
                                       g.ctypes.data_as(C.c_void_p)))
    return g


# ------------------------------------------------------ surrogate network ---

def mdlg_mlp_create(params, max_batch, stream=None) -> C.c_void_p:
    p = _host(params, np.float32, MLP_NPARAMS)
    h = C.c_void_p()
    _abi.check(_abi.lib().mdlg_mlp_create(C.byref(h), p.ctypes.data_as(C.c_void_p), int(max_batch), _stream(stream)))
    return h


def mdlg_mlp_params(h, stream=None) -> np.ndarray:
    out = np.zeros(MLP_NPARAMS, dtype=np.float32)
    _abi.check(_abi.lib().mdlg_mlp_params(h, out.ctypes.data_as(C.c_void_p), _stream(stream)))
    return out


def mdlg_mlp_forward(h, x, g_out=None, stream=None):
    torch = _torch()
    B = int(x.shape[0])
    if g_out is None:
        g_out = torch.empty((B, 49), dtype=torch.float32, device=x.device)
    _abi.check(_abi.lib().mdlg_mlp_forward(h, _dev(x, torch.float32, (B, 6), "x"), B,
                                           _dev(g_out, torch.float32, (B, 49), "g_out"), _stream(stream)))
    return g_out


def mdlg_mlp_gradient(h, x, target, stream=None):
    """Returns (loss tensor [1], grad tensor [NPARAMS]) on the device."""
    torch = _torch()
    B = int(x.shape[0])
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    grad = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=x.device)
    _abi.check(_abi.lib().mdlg_mlp_gradient(h, _dev(x, torch.float32, (B, 6), "x"),
                                            _dev(target, torch.float32, (B, 49), "target"), B,
                                            _dev(loss, torch.float32), _dev(grad, torch.float32), _stream(stream)))
    return loss, grad


def mdlg_mlp_train_step(h, x, target, lr, loss=None, stream=None):
    torch = _torch()
    B = int(x.shape[0])
    _abi.check(_abi.lib().mdlg_mlp_train_step(h, _dev(x, torch.float32, (B, 6), "x"),
                                              _dev(target, torch.float32, (B, 49), "target"), B, float(lr),
                                              _dev(loss, torch.float32, (1,), "loss"), _stream(stream)))
    return loss


def mdlg_feq_surrogate(h, x, a2, lam, tol=1e-3, stream=None):
    """Returns (g [49] float64, used_fallback bool, max |g_net - g_wsg|)."""
    xx = _host(x, np.float64, 6)
    g = np.zeros(49)
    fb = C.c_int32(0)
    err = C.c_double(0.0)
    _abi.check(_abi.lib().mdlg_feq_surrogate(h, xx.ctypes.data_as(C.c_void_p), float(a2), float(lam), float(tol),
                                             g.ctypes.data_as(C.c_void_p), C.byref(fb), C.byref(err),
                                             _stream(stream)))
    return g, bool(fb.value), float(err.value)


def mdlg_mlp_destroy(h):
    _abi.lib().mdlg_mlp_destroy(h)


def mdlg_moment_table_create(samples, dims=(6, 8, 12), smooth=1e-3, branch=2, lo=None, hi=None):
    """samples [n, 5] = (phi, kT, dt_cg/dx, a2, r); lo, hi (phi, kT, dt_cg/dx):
    the grid's box (default: the samples' bounding box); returns the handle."""
    ss = np.ascontiguousarray(samples, dtype=np.float64)
    if ss.ndim != 2 or ss.shape[1] != 5 or ss.shape[0] < 1:
        raise ValueError(f"samples: expected shape (n >= 1, 5), got {ss.shape}")
    dd = _host(dims, np.int32, 3)
    if (lo is None) != (hi is None):
        raise ValueError("give both lo and hi, or neither")
    ll = None if lo is None else _host(lo, np.float64, 3)
    hh = None if hi is None else _host(hi, np.float64, 3)
    h = C.c_void_p()
    _abi.check(_abi.lib().mdlg_moment_table_create(
        C.byref(h), ss.ctypes.data_as(C.c_void_p), ss.shape[0], dd.ctypes.data_as(C.c_void_p),
        None if ll is None else ll.ctypes.data_as(C.c_void_p), None if hh is None else hh.ctypes.data_as(C.c_void_p),
        float(smooth), int(branch)))
    return h


def mdlg_moment_table_eval(t, x):
    """x = (phi, kT, dt_cg/dx) -> (a2, lambda, r)."""
    xx = _host(x, np.float64, 3)
    a2, lam, r = C.c_double(), C.c_double(), C.c_double()
    _abi.check(_abi.lib().mdlg_moment_table_eval(t, xx.ctypes.data_as(C.c_void_p), C.byref(a2), C.byref(lam),
                                                 C.byref(r)))
    return a2.value, lam.value, r.value


def mdlg_moment_table_info(t):
    """Returns (dims [3], lo [3], hi [3], nodes [P, 2] = (ln a2, r))."""
    dims = np.zeros(3, np.int32)
    lo, hi = np.zeros(3), np.zeros(3)
    _abi.check(_abi.lib().mdlg_moment_table_info(t, dims.ctypes.data_as(C.c_void_p), lo.ctypes.data_as(C.c_void_p),
                                                 hi.ctypes.data_as(C.c_void_p), None))
    nodes = np.zeros((int(np.prod(dims)), 2))
    _abi.check(_abi.lib().mdlg_moment_table_info(t, None, None, None, nodes.ctypes.data_as(C.c_void_p)))
    return dims, lo, hi, nodes


def mdlg_moment_table_destroy(t):
    _abi.lib().mdlg_moment_table_destroy(t)


def mdlg_feq_surrogate_table(h, table, x, tol=1e-3, stream=None):
    """Returns (g [49] float64, used_fallback bool, max |g_net - g_wsg|, a2, lambda)."""
    xx = _host(x, np.float64, 6)
    g = np.zeros(49)
    fb = C.c_int32(0)
    err, a2, lam = C.c_double(0.0), C.c_double(0.0), C.c_double(0.0)
    _abi.check(_abi.lib().mdlg_feq_surrogate_table(h, table, xx.ctypes.data_as(C.c_void_p), float(tol),
                                                   g.ctypes.data_as(C.c_void_p), C.byref(fb), C.byref(err),
                                                   C.byref(a2), C.byref(lam), _stream(stream)))
    return g, bool(fb.value), float(err.value), a2.value, lam.value


class MomentTable:
    """Owns one mdlg_moment_table handle (host memory only)."""

    def __init__(self, samples, dims=(6, 8, 12), smooth=1e-3, branch=2, lo=None, hi=None):
        self.handle = mdlg_moment_table_create(samples, dims, smooth, branch, lo, hi)

    def close(self):
        if getattr(self, "handle", None):
            mdlg_moment_table_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __call__(self, x):
        return mdlg_moment_table_eval(self.handle, x)

    def info(self):
        return mdlg_moment_table_info(self.handle)


class SurrogateMLP:
    """Owns one mdlg_mlp handle."""

    def __init__(self, params, max_batch, stream=None):
        self.stream = stream
        self.max_batch = int(max_batch)
        self.handle = mdlg_mlp_create(params, max_batch, stream)

    def close(self):
        if getattr(self, "handle", None):
            mdlg_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        return mdlg_mlp_params(self.handle, self.stream)

    def forward(self, x):
        return mdlg_mlp_forward(self.handle, x, stream=self.stream)

    def gradient(self, x, target):
        return mdlg_mlp_gradient(self.handle, x, target, self.stream)

    def train_step(self, x, target, lr, loss=None):
        return mdlg_mlp_train_step(self.handle, x, target, lr, loss, self.stream)

    def feq(self, x, a2, lam, tol=1e-3):
        return mdlg_feq_surrogate(self.handle, x, a2, lam, tol, self.stream)

    def feq_table(self, x, table: "MomentTable", tol=1e-3):
        return mdlg_feq_surrogate_table(self.handle, table.handle, x, tol, self.stream)


# ------------------------------------------------------ convenience class ---

@dataclass
class CGAccumulators:
    counts: object    # torch int64 [n_rep, 50]
    moments: object   # torch float64 [n_rep, 5]
    cell_acc: object  # torch int32 or None
    lattices: list
    s_cg: int
    system: "LJSystem"

    @property
    def events(self) -> int:
        return lj_md_info(self.system.handle)["events_done"]


class LJSystem:
    """Owns one lj_md handle (one system or a batch of replicas)."""

    def __init__(self, pos0, vel0, box_l=None, params=None, stream=None, **kw):
        if params is None:
            params = [lj_params(pos0.shape[0], box_l, **kw)]
        elif isinstance(params, LJParams):
            params = [params]
        self.params = list(params)
        self.n_rep = len(self.params)
        self.n_total = sum(p.n for p in self.params)
        self.stream = stream
        if self.n_rep == 1:
            self.handle = lj_md_init(self.params[0], pos0, vel0, stream)
        else:
            self.handle = lj_md_init_batch(self.params, pos0, vel0, stream)
        self.cg = None

    def close(self):
        if self.handle:
            lj_md_destroy(self.handle)
            self.handle = None

    def save(self, path):
        lj_md_save(self.handle, path, self.stream)

    @classmethod
    def load(cls, path, stream=None):
        """A system resumed from a file written by save()."""
        obj = cls.__new__(cls)
        obj.handle = lj_md_load(path, stream)
        obj.stream = stream
        info = lj_md_info(obj.handle)
        obj.n_rep = info["n_rep"]
        obj.n_total = info["n_total"]
        obj.params = None
        obj.cg = None
        return obj

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def attach_cg(self, lx, s_cg, u=(0.0, 0.0), cell_acc=False) -> CGAccumulators:
        torch = _torch()
        lxs = list(lx) if hasattr(lx, "__len__") else [lx] * self.n_rep
        us = list(u) if (hasattr(u, "__len__") and len(u) == self.n_rep and hasattr(u[0], "__len__")) \
            else [u] * self.n_rep
        lats = [Lattice(lx=int(l), reserved=0, u=(C.c_double * 2)(float(v[0]), float(v[1])))
                for l, v in zip(lxs, us)]
        counts = torch.zeros((self.n_rep, 50), dtype=torch.int64, device="cuda")
        moments = torch.zeros((self.n_rep, 5), dtype=torch.float64, device="cuda")
        cacc = None
        if cell_acc:
            cacc = torch.zeros(sum(49 * l * l for l in lxs), dtype=torch.int32, device="cuda")
        lj_md_cg_attach(self.handle, s_cg, lats, counts, moments, cacc, self.stream)
        self.cg = CGAccumulators(counts, moments, cacc, lats, s_cg, self)
        return self.cg

    def detach_cg(self):
        lj_md_cg_detach(self.handle)
        self.cg = None

    def step(self, nsteps):
        lj_md_step(self.handle, nsteps, self.stream)

    def step_timed(self, nunits, sample_every=1):
        return lj_md_step_timed(self.handle, nunits, self.stream, sample_every)

    def state(self):
        torch = _torch()
        pos = torch.empty((self.n_total, 2), dtype=torch.float64, device="cuda")
        vel = torch.empty_like(pos)
        img = torch.empty((self.n_total, 2), dtype=torch.int32, device="cuda")
        lj_md_get_state(self.handle, pos, vel, img, self.stream)
        return pos, vel, img

    def forces(self):
        torch = _torch()
        f = torch.empty((self.n_total, 2), dtype=torch.float64, device="cuda")
        lj_md_forces(self.handle, f, self.stream)
        return f

    def energy(self):
        return lj_md_energy(self.handle, self.stream)

    def check(self):
        lj_md_check(self.handle, self.stream)

    def info(self):
        return lj_md_info(self.handle)
