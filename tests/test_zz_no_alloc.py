"""mdlg_coarse_grain_noalloc (no device allocation, fixed scratch) against
mdlg_coarse_grain on the same snapshots, through the C ABI: counts, moments,
dense n_i(x, t) and per-cell accumulators bitwise equal, on two calls in a
row (the second with fewer particles, so stale partials of the first would
show), and the size limit refused before any launch."""
import numpy as np
import pytest

import mdlg_inputs as mi

pytestmark = pytest.mark.gpu


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _snapshots(n, L, seed, step=1.7):
    """Two snapshots of a seeded random walk (wrapped positions and image counts)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p0 = rng.uniform(0.0, L, (n, 2))
    d = rng.normal(0.0, step, (n, 2))
    u = p0 + d
    img = np.floor(u / L).astype(np.int32)
    p1 = u - L * img
    p1[p1 >= L] = 0.0
    return p0, np.zeros((n, 2), np.int32), p1, img


def _run(m, noalloc, lx, L, p0, i0, p1, i1, k_prev, k_cur, u):
    import torch
    counts = torch.zeros(50, dtype=torch.int64, device="cuda")
    moments = torch.zeros(5, dtype=torch.float64, device="cuda")
    n_event = torch.full((49, lx, lx), 7, dtype=torch.int32, device="cuda")
    cell_acc = torch.zeros((49, lx, lx), dtype=torch.int32, device="cuda")
    m.mdlg_coarse_grain(lx, L, _cuda(p0), _cuda(p1), counts, moments, _cuda(i0), _cuda(i1), k_prev, k_cur, u,
                        n_event, cell_acc, noalloc=noalloc)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (counts, moments, n_event, cell_acc)]


@pytest.mark.parametrize("sizes", [(300_001, 4_097), (1 << 20, 1)])
def test_noalloc_equals_allocating_entry_point(sizes):
    import paper_2101_01160_amd as m
    lx, L = 64, 200.0
    for call, n in enumerate(sizes):
        print(f"noalloc call {call}: n={n}", flush=True)
        p0, i0, p1, i1 = _snapshots(n, L, seed=11 + call)
        ref = _run(m, False, lx, L, p0, i0, p1, i1, 3, 4, (0.1, -0.05))
        got = _run(m, True, lx, L, p0, i0, p1, i1, 3, 4, (0.1, -0.05))
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
        assert int(got[0].sum()) == n


def test_noalloc_from_md_snapshots():
    """Snapshots of the GPU MD itself (the paper's gas at phi = 0.0784, kT = 20)."""
    import torch

    import paper_2101_01160_amd as m
    n, lx = 20000, 50
    pos0, vel0, L = mi.initial_state(n, 0.0784, 20.0, 5)
    sysm = m.LJSystem(_cuda(pos0), _cuda(vel0), box_l=L)
    sysm.step(400)
    p1, _, i1 = (t.cpu().numpy() for t in sysm.state())
    sysm.close()
    torch.cuda.synchronize()
    i0 = np.zeros((n, 2), np.int32)
    ref = _run(m, False, lx, L, pos0, i0, p1, i1, 0, 1, (0.0, 0.0))
    got = _run(m, True, lx, L, pos0, i0, p1, i1, 0, 1, (0.0, 0.0))
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_noalloc_refuses_sizes_beyond_its_scratch():
    import torch

    import paper_2101_01160_amd as m
    lat = m.Lattice(lx=8, reserved=0)
    counts = torch.zeros(50, dtype=torch.int64, device="cuda")
    dummy = torch.zeros((1, 2), dtype=torch.float64, device="cuda")
    # n beyond the limit is refused on the host (the pointers are never read)
    st = m._abi.lib().mdlg_coarse_grain_noalloc(
        m._abi.C.byref(lat), 10.0, m.NOALLOC_MAX_N + 1, m._abi.C.c_void_p(dummy.data_ptr()), None, 0,
        m._abi.C.c_void_p(dummy.data_ptr()), None, 1, m._abi.C.c_void_p(counts.data_ptr()), None, None, None,
        m._abi.C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == -1
    assert "exceeds" in m._abi.lib().mdlg_last_error().decode()
    assert int(counts.sum().item()) == 0
