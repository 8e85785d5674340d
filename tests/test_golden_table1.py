"""Table 1 of the paper (MD initialisation parameters) read as this library
reads it: every row describes the same box, L = dx * lx = 1000 sigma (the
5.5 / 180 row has dx = 1000/180 = 5.55..., printed rounded); the MD output
frequency is the number of MD steps per coarse step, dt_cg / 1e-4; the total
MD time is 2000 coarse iterations of dt_cg (the table caption)."""
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def rows():
    out = []
    for ln in open(os.path.join(HERE, "golden", "table1.txt")):
        ln = ln.strip()
        if ln and not ln.startswith("#"):
            out.append([float(x) for x in ln.split()])
    return np.array(out)


def test_table_has_twelve_rows():
    assert rows().shape == (12, 5)


@pytest.mark.parametrize("i", range(12))
def test_row_identities(i):
    dt_cg, dx, lx, freq, total = rows()[i]
    # one box for every lattice: L = dx * lx = 1000 sigma (dx printed to 2-3 digits)
    assert dx * lx == pytest.approx(1000.0, rel=1.2e-2)
    # MD steps per coarse step with dt = 1e-4 tau_LJ
    assert freq == pytest.approx(dt_cg / 1e-4, abs=0.6)
    # 2000 coarse iterations
    assert total == pytest.approx(2000.0 * dt_cg, rel=1e-9)


def test_coarse_time_grows_with_lattice_spacing():
    r = rows()
    assert np.all(np.diff(r[:, 1]) > 0) and np.all(np.diff(r[:, 0]) > 0)
    # the coarse time step scales faster than linearly with dx over the table
    slope = np.polyfit(np.log(r[:, 1]), np.log(r[:, 0]), 1)[0]
    assert 1.0 < slope < 2.0


def test_benchmark_sweep_uses_the_table():
    """The paper-regime benchmark runs exactly these rows."""
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    import bench
    r = rows()
    assert len(bench.TABLE1) == 12
    for (dt_cg, dx, lx, freq), ref in zip(bench.TABLE1, r):
        assert (dt_cg, lx, freq) == (ref[0], int(ref[2]), int(ref[3]))
        assert dx == pytest.approx(ref[1], rel=1e-15)
