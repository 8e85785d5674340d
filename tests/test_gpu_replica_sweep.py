"""The batching configuration at its full shape, against single runs and the oracle.

256 replicas of the (phi, kT, seed) sweep: N log-uniform in [4096, 262144]
(18.6M particles in all), phi in {0.0784, 0.2, 0.4} x kT in {1, 5, 20},
lattices of ~2 sigma cells, a coarse-graining event every 50 MD steps,
launch parameters from the autotuner, 100 MD steps as one batch.  Sampled
replicas (the smallest, the largest and the first of each area fraction)
equal the same replica run alone with the same launch parameters, bit for
bit in positions, velocities, images, counts and moment sums; the smallest
also matches the oracle (positions and velocities within 1e-10 relative,
images and counts exact).
"""
import numpy as np
import pytest

import mdlg_inputs as mi
from oracle import md as omd

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def test_replica_sweep_batch_equals_single_runs_and_oracle():
    import torch

    import paper_2101_01160_amd as m
    s_cg, nsteps = 50, 100
    specs = mi.replica_sweep(256)
    states = [mi.initial_state(sp.n, sp.phi, sp.kT, sp.seed) for sp in specs]
    sizes = [sp.n for sp in specs]
    print(f"replica sweep: {len(specs)} replicas, {sum(sizes)} particles", flush=True)
    tpos = torch.from_numpy(np.concatenate([st[0] for st in states])).cuda()
    tvel = torch.from_numpy(np.concatenate([st[1] for st in states])).cuda()
    params = [m.lj_params(sp.n, sp.L) for sp in specs]
    lats = [m.Lattice(lx=sp.lx, reserved=0) for sp in specs]
    bparams, _ = m.lj_md_autotune(params, tpos, tvel, s_cg, lats, use_cache=False)
    print(f"replica sweep: tuned step_kernel={bparams[0].step_kernel} block_size={bparams[0].block_size}",
          flush=True)
    batch = m.LJSystem(tpos, tvel, params=bparams)
    acc = batch.attach_cg([sp.lx for sp in specs], s_cg)
    info = batch.info()
    K, spl = info["rebuild_every"], info["steps_per_launch"]
    batch.step(nsteps)
    torch.cuda.synchronize()
    batch.check()
    assert acc.events == nsteps // s_cg
    bp, bv, bi = (_np(t) for t in batch.state())
    bc, bm = _np(acc.counts), _np(acc.moments)
    batch.close()
    del tpos, tvel
    offs = np.concatenate([[0], np.cumsum(sizes)])
    # every replica's counts add up to its particles times the events
    assert np.array_equal(bc.sum(axis=1), np.asarray(sizes) * (nsteps // s_cg))

    sample = {int(np.argmin(sizes)), int(np.argmax(sizes))}
    sample |= {next(r for r, sp in enumerate(specs) if sp.phi == phi) for phi in (0.0784, 0.2, 0.4)}
    for r in sorted(sample):
        sp, (p0, v0, L) = specs[r], states[r]
        print(f"replica {r}: n={sp.n} phi={sp.phi} kT={sp.kT}", flush=True)
        p = m.LJParams.from_buffer_copy(bparams[r])
        p.rebuild_every = K
        p.fuse_steps = spl
        single = m.LJSystem(torch.from_numpy(p0).cuda(), torch.from_numpy(v0).cuda(), params=[p])
        assert single.info()["steps_per_launch"] == spl
        sacc = single.attach_cg(sp.lx, s_cg)
        single.step(nsteps)
        torch.cuda.synchronize()
        single.check()
        sp_, sv, si = (_np(t) for t in single.state())
        a, b = offs[r], offs[r + 1]
        assert np.array_equal(bp[a:b], sp_)
        assert np.array_equal(bv[a:b], sv)
        assert np.array_equal(bi[a:b], si)
        assert np.array_equal(bc[r], _np(sacc.counts)[0])
        assert np.array_equal(bm[r], _np(sacc.moments)[0])
        single.close()

    r = int(np.argmin(sizes))
    sp, (p0, v0, L) = specs[r], states[r]
    print(f"replica {r} against the oracle", flush=True)
    oacc = omd.CGAccum(sp.lx)
    po, vo, io, _ = omd.md_run(p0.copy(), v0.copy(), np.zeros((sp.n, 2), np.int64), L, nsteps, cg=oacc,
                               s_cg=s_cg)
    a, b = offs[r], offs[r + 1]
    assert np.array_equal(bi[a:b], io)
    up, uo = bp[a:b] + L * bi[a:b], po + L * io
    assert np.max(np.abs(up - uo)) <= 1e-10 * np.abs(uo).max()
    assert np.max(np.abs(bv[a:b] - vo)) <= 1e-10 * np.abs(vo).max()
    assert np.array_equal(bc[r], oacc.counts)
