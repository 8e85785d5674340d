"""Training data, training and evaluation of the f_eq surrogate network.

Every number is produced on the GPU by the library: batched LJ molecular
dynamics (lj_md_*) generates the trajectories, mdlg_coarse_grain_series turns
stored snapshots into occupation counts for many coarse-graining times and
lattice drifts at once (Eq.(n_i)), and the network (mdlg_mlp_*) trains on the
measured equilibria g_i = f_i^eq / rho (Eq.(theory_feq)) with the
Kullback-Leibler loss of Eq.(kullback_leibler).  The closed forms (host FP64:
mdlg_feq_wsg with lambda from Eq.(lambda_eq)) serve as the guard.

Sample design (the paper's dilute-to-moderate LJ gas, lattice spacing
dx = L / round(L / 2) ~ 2 sigma):
  * replicas: phi ~ U(0.05, 0.4), kT ~ U(1, 20), N particles each, in groups
    that share one batched MD handle and one set of drifts;
  * coarse-graining time dt_cg = lag * stride * dt for lags in snapshots;
    every snapshot pair at that lag is one event, on a lattice whose origin
    moves along a low-discrepancy sequence from pair to pair (translation
    averaging: unbiased for a homogeneous gas, and it decorrelates the
    cell-crossing events of overlapping pairs);
  * drifts u (cells per coarse step): (0, 0) and |u| = u_max sqrt(U(0, 1)),
    angle U(0, 2 pi), drawn per group;
  * network inputs (phi, kT, dt_cg / dx, |u|, cos, sin), direction (1, 0) at
    u = 0; targets the measured g_i (49 values) of each (replica, lag, drift).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

import mdlg_inputs as mi

from . import (LJParams, MomentTable, SurrogateMLP, lj_md_destroy, lj_md_get_state, lj_md_init_batch, lj_md_step,
               mdlg_coarse_grain_series, mdlg_feq_measured, mdlg_feq_wsg, mdlg_lambda_from_moments, mdlg_moments)

DEFAULT_LAGS = (1, 2, 3, 4, 6, 8, 10, 13, 16, 20)


@dataclass
class SurrogateData:
    X: np.ndarray         # [M, 6] network inputs
    G: np.ndarray         # [M, 49] measured g_i
    overflow: np.ndarray  # [M] fraction beyond |v_a| <= 3
    a2: np.ndarray        # [M] measured a^2 (lattice units)
    lam: np.ndarray       # [M] lambda from the displacement moments
    r: np.ndarray         # [M] kurtosis ratio mu4 / (3 mu2^2) of the displacements
    rep: np.ndarray       # [M] replica id (for splits without leakage)
    u: np.ndarray         # [M, 2] drift, cells per coarse step
    samples: np.ndarray   # [M] particle events behind each g
    timing: dict = field(default_factory=dict)

    def __len__(self):
        return self.X.shape[0]

    def subset(self, idx):
        return SurrogateData(self.X[idx], self.G[idx], self.overflow[idx], self.a2[idx], self.lam[idx], self.r[idx],
                             self.rep[idx], self.u[idx], self.samples[idx], dict(self.timing))


def lattice_origins(n_snap):
    """Lattice origins (cells) of the pairs starting at each snapshot: the
    additive recurrence of the plastic number (Roberts' R2 sequence), which
    covers the unit cell evenly, so that overlapping pairs sample independent
    in-cell positions."""
    g = 1.32471795724474602596
    p = np.arange(n_snap, dtype=np.float64)[:, None]
    return np.mod(0.5 + p * np.array([1.0 / g, 1.0 / (g * g)]), 1.0)


def drift_set(n_u, u_max, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    r = u_max * np.sqrt(rng.uniform(0.0, 1.0, n_u))
    th = rng.uniform(0.0, 2.0 * math.pi, n_u)
    u = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
    u[0] = 0.0
    return u


def generate(n_groups=4, reps_per_group=80, n=65536, n_snap=401, stride=10, equil=3000, lags=DEFAULT_LAGS,
             n_u=16, u_max=0.2, dt=1e-4, seed=12345, log=None) -> SurrogateData:
    """Run the sample design above on the GPU; returns the measured equilibria."""
    import torch
    lags = tuple(int(l) for l in lags)
    out = {k: [] for k in ("X", "G", "overflow", "a2", "lam", "r", "rep", "u", "samples")}
    t_md = t_cg = 0.0
    for g in range(n_groups):
        specs = mi.surrogate_sweep(reps_per_group, seed=seed + g, n=n)
        pos0, vel0, params = [], [], []
        for s in specs:
            p, v, L = mi.initial_state(s.n, s.phi, s.kT, s.seed)
            pos0.append(p)
            vel0.append(v)
            params.append(LJParams(n=s.n, box_l=L, dt=dt, rc=2.5, eps=1.0, energy_shift=1, force_bits=64,
                                   skin=0.0, rebuild_every=0, block_size=0, step_kernel=0, gather_batch=0))
        n_tot = sum(s.n for s in specs)
        pos_d = torch.from_numpy(np.concatenate(pos0)).cuda()
        vel_d = torch.from_numpy(np.concatenate(vel0)).cuda()
        snaps = torch.empty((n_snap, n_tot, 2), dtype=torch.float64, device="cuda")
        imgs = torch.empty((n_snap, n_tot, 2), dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = lj_md_init_batch(params, pos_d, vel_d)
        try:
            lj_md_step(h, equil)
            for p in range(n_snap):
                if p:
                    lj_md_step(h, stride)
                lj_md_get_state(h, snaps[p], None, imgs[p])
            torch.cuda.synchronize()
        finally:
            lj_md_destroy(h)
        t1 = time.perf_counter()
        del pos_d, vel_d
        u = drift_set(n_u, u_max, seed * 7 + g)
        offsets = np.concatenate([[0], np.cumsum([s.n for s in specs])])
        box = np.array([p.box_l for p in params])
        lx = np.array([s.lx for s in specs], dtype=np.int32)
        counts = torch.zeros((len(specs), len(lags), n_u, 50), dtype=torch.int64, device="cuda")
        moments = torch.zeros((len(specs), len(lags), 5), dtype=torch.float64, device="cuda")
        mdlg_coarse_grain_series(offsets, box, lx, snaps, imgs, lags, u, counts, moments,
                                 lattice_offset=lattice_origins(n_snap))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_md += t1 - t0
        t_cg += t2 - t1
        del snaps, imgs
        counts = counts.cpu().numpy()
        moments = moments.cpu().numpy()
        for r, s in enumerate(specs):
            dx = box[r] / lx[r]
            for si, l in enumerate(lags):
                pairs = n_snap - l
                mu2, mu4, a2 = mdlg_moments(moments[r, si], dx)
                lam, kr = mdlg_lambda_from_moments(mu2, mu4, 2)
                for t in range(n_u):
                    um = float(np.hypot(*u[t]))
                    c, sn = (u[t] / um) if um > 0 else (1.0, 0.0)
                    out["X"].append((s.phi, s.kT, l * stride * dt / dx, um, c, sn))
                    g_meas, ovf = mdlg_feq_measured(counts[r, si, t], s.n, pairs)
                    out["G"].append(g_meas)
                    out["overflow"].append(ovf)
                    out["a2"].append(a2)
                    out["lam"].append(lam)
                    out["r"].append(kr)
                    out["rep"].append(g * reps_per_group + r)
                    out["u"].append(u[t])
                    out["samples"].append(s.n * pairs)
        if log:
            log(f"surrogate data: group {g + 1}/{n_groups} ({len(specs)} replicas x {n} particles): "
                f"MD {t1 - t0:.2f} s, coarse-graining {t2 - t1:.3f} s")
    d = SurrogateData(*(np.asarray(out[k], dtype=np.float64) for k in ("X", "G", "overflow", "a2", "lam", "r")),
                      np.asarray(out["rep"], dtype=np.int64), np.asarray(out["u"], dtype=np.float64),
                      np.asarray(out["samples"], dtype=np.int64))
    d.timing = {"md_s": t_md, "cg_s": t_cg,
                "particle_steps": float(n_groups * reps_per_group * n * (equil + (n_snap - 1) * stride)),
                "particle_snapshots": float(n_groups * reps_per_group * n * n_snap)}
    return d


def split_by_replica(data: SurrogateData, seed=0, frac=(0.8, 0.1, 0.1)):
    """Index arrays (train, val, test) with every replica in exactly one part."""
    reps = np.unique(data.rep)
    rng = np.random.Generator(np.random.PCG64(seed))
    reps = rng.permutation(reps)
    n_tr = int(round(frac[0] * reps.size))
    n_va = int(round(frac[1] * reps.size))
    parts = (reps[:n_tr], reps[n_tr:n_tr + n_va], reps[n_tr + n_va:])
    return tuple(np.flatnonzero(np.isin(data.rep, p)) for p in parts)


def train(data: SurrogateData, idx, steps=4000, batch=4096, lr=2e-3, lr_final=2e-5, init_seed=0, seed=0,
          val_idx=None, val_every=500, log=None, average_tail=0.0, average_every=100):
    """Adam on minibatches drawn without replacement per epoch; cosine learning rate.
    With average_tail > 0 the returned network holds the mean of the
    parameters taken every `average_every` steps over that last fraction of
    the steps (weight averaging: it removes most of the minibatch noise the
    final iterate carries).  Returns (network, history dict)."""
    import torch
    net = SurrogateMLP(mi.mlp_init(init_seed).astype(np.float32), max(batch, 1))
    X = torch.from_numpy(data.X[idx].astype(np.float32)).cuda()
    # targets: the measured g_i as they are (in this regime no displacement
    # leaves D2Q49, so they sum to one like the network's softmax)
    R = torch.from_numpy(data.G[idx].astype(np.float32)).cuda()
    m = X.shape[0]
    batch = min(batch, m)
    rng = np.random.Generator(np.random.PCG64(seed))
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = {"step": [], "loss": [], "val_max_err": []}
    perm, pos = torch.from_numpy(rng.permutation(m)).cuda(), 0
    avg_from = steps - int(round(average_tail * steps)) if average_tail > 0 else steps
    avg_sum, avg_n = None, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        if pos + batch > m:
            perm, pos = torch.from_numpy(rng.permutation(m)).cuda(), 0
        sel = perm[pos:pos + batch]
        pos += batch
        xb = X.index_select(0, sel)
        rb = R.index_select(0, sel)
        lr_k = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * k / max(1, steps - 1)))
        net.train_step(xb, rb, lr_k, loss)
        if k >= avg_from and (k + 1 - avg_from) % average_every == 0:
            p = net.params().astype(np.float64)
            avg_sum = p if avg_sum is None else avg_sum + p
            avg_n += 1
        if (k + 1) % val_every == 0 or k + 1 == steps:
            hist["step"].append(k + 1)
            hist["loss"].append(float(loss.cpu()[0]))
            if val_idx is not None:
                hist["val_max_err"].append(evaluate(net, data, val_idx)["max_err"])
            if log:
                v = f" val max|dg| {hist['val_max_err'][-1]:.2e}" if val_idx is not None else ""
                log(f"surrogate train: step {k + 1}/{steps} loss {hist['loss'][-1]:.3e}{v}")
    if avg_n:
        net = SurrogateMLP((avg_sum / avg_n).astype(np.float32), max(batch, 1))
        hist["averaged"] = avg_n
    torch.cuda.synchronize()
    hist["train_s"] = time.perf_counter() - t0
    return net, hist


def predict(net: SurrogateMLP, X):
    import torch
    out = []
    for a in range(0, X.shape[0], net.max_batch):
        x = torch.from_numpy(np.ascontiguousarray(X[a:a + net.max_batch], dtype=np.float32)).cuda()
        out.append(net.forward(x).cpu().numpy().astype(np.float64))
    return np.concatenate(out)


def moment_table(data: SurrogateData, idx, dims=(6, 8, 12), smooth=1e-3, box=None):
    """The library's moment table fitted to the measured (a^2, r) of the given
    samples (one row per replica and coarse-graining time), for the guard at
    points where no trajectory exists.  box = (lo, hi) over (phi, kT,
    dt_cg/dx), the parameter range to cover (default: the samples' own)."""
    _, first = np.unique(np.stack([data.rep[idx], data.X[idx, 2]], axis=1), axis=0, return_index=True)
    sel = np.asarray(idx)[np.sort(first)]
    rows = np.stack([data.X[sel, 0], data.X[sel, 1], data.X[sel, 2], data.a2[sel], data.r[sel]], axis=1)
    lo, hi = (None, None) if box is None else box
    return MomentTable(rows, dims=dims, smooth=smooth, branch=2, lo=lo, hi=hi)


def parameter_box(data: SurrogateData):
    """The design's parameter range over (phi, kT, dt_cg/dx) as its inputs
    span it (no measured value enters)."""
    return data.X[:, :3].min(axis=0), data.X[:, :3].max(axis=0)


def wsg_table(data: SurrogateData, idx, table: MomentTable | None = None):
    """Poisson-WSG equilibrium of each sample: from its measured a^2 and lambda,
    or, given a table, from the table's a^2 and lambda at (phi, kT, dt_cg/dx)."""
    if table is None:
        return np.stack([mdlg_feq_wsg(data.a2[i], data.lam[i], data.u[i]) for i in idx])
    out = []
    for i in idx:
        a2, lam, _ = table(data.X[i, :3])
        out.append(mdlg_feq_wsg(a2, lam, data.u[i]))
    return np.stack(out)


def evaluate(net: SurrogateMLP, data: SurrogateData, idx, tol=1e-3, with_guard=False, table=None):
    """Errors of the network against the measured g (max over the 49 values per
    sample); with_guard adds the WSG comparison and the fallback rate at tol,
    with the measured moments of each sample and, given a moment table, with
    the table's (the guard that needs no trajectory)."""
    g = predict(net, data.X[idx])
    err = np.abs(g - data.G[idx]).max(axis=1)
    res = {"max_err": float(err.max()), "mean_err": float(err.mean()), "p99_err": float(np.quantile(err, 0.99)),
           "frac_below_tol": float(np.mean(err <= tol)), "n": int(len(idx))}
    if with_guard:
        for key, tab in (("", None), ("table_", table)):
            if key and tab is None:
                continue
            w = wsg_table(data, idx, tab)
            dev_wsg = np.abs(g - w).max(axis=1)
            fallback = dev_wsg > tol
            final = np.where(fallback[:, None], w, g)
            e_final = np.abs(final - data.G[idx]).max(axis=1)
            e_wsg = np.abs(w - data.G[idx]).max(axis=1)
            res.update({key + "fallback_rate": float(fallback.mean()), key + "guarded_max_err": float(e_final.max()),
                        key + "guarded_mean_err": float(e_final.mean()), key + "wsg_max_err": float(e_wsg.max()),
                        key + "wsg_mean_err": float(e_wsg.mean())})
    return res
