"""The binding refuses buffers whose dtype or shape does not match the handle
before anything reaches the library (no GPU: the handle's extents are
supplied in place of lj_md_info, and CPU tensors stand in for device ones)."""
import ctypes as C

import pytest


@pytest.fixture
def fake_handle(monkeypatch):
    import paper_2101_01160_amd as m

    def info(h):
        return {"n_rep": 3, "n_total": 1000}
    monkeypatch.setattr(m, "lj_md_info", info)
    return C.c_void_p(1)


def _t(shape, dtype):
    import torch
    return torch.zeros(shape, dtype=dtype)


@pytest.mark.parametrize("which", ["pos", "vel", "img"])
def test_get_state_refuses_undersized_buffers(fake_handle, which):
    import torch

    import paper_2101_01160_amd as m
    kw = {"pos": _t((1000, 2), torch.float64), "vel": _t((1000, 2), torch.float64),
          "img": _t((1000, 2), torch.int32)}
    kw[which] = kw[which][:999]
    with pytest.raises(ValueError, match="shape"):
        m.lj_md_get_state(fake_handle, **kw, stream=0)


def test_forces_refuse_undersized_buffer(fake_handle):
    import torch

    import paper_2101_01160_amd as m
    with pytest.raises(ValueError, match="shape"):
        m.lj_md_forces(fake_handle, _t((1000, 1), torch.float64), stream=0)
    with pytest.raises(ValueError, match="dtype"):
        m.lj_md_forces(fake_handle, _t((1000, 2), torch.float32), stream=0)


def test_correctly_sized_host_buffer_is_still_refused(fake_handle):
    import torch

    import paper_2101_01160_amd as m
    with pytest.raises(ValueError, match="GPU"):
        m.lj_md_forces(fake_handle, _t((1000, 2), torch.float64), stream=0)


@pytest.mark.parametrize("field,shape", [("counts", (3, 49)), ("counts", (1, 50)), ("moments", (3, 4)),
                                         ("cell_acc", (49 * 100,))])
def test_cg_attach_refuses_wrong_accumulators(fake_handle, field, shape):
    import torch

    import paper_2101_01160_amd as m
    lats = [m.Lattice(lx=10, reserved=0, u=(C.c_double * 2)(0.0, 0.0)) for _ in range(3)]
    kw = {"counts": _t((3, 50), torch.int64), "moments": _t((3, 5), torch.float64),
          "cell_acc": _t((3 * 49 * 100,), torch.int32)}
    kw[field] = _t(shape, kw[field].dtype)
    with pytest.raises(ValueError, match="shape"):
        m.lj_md_cg_attach(fake_handle, 10, lats, kw["counts"], kw["moments"], kw["cell_acc"], stream=0)


def test_cg_attach_needs_one_lattice_per_replica(fake_handle):
    import torch

    import paper_2101_01160_amd as m
    lats = [m.Lattice(lx=10, reserved=0, u=(C.c_double * 2)(0.0, 0.0))]
    with pytest.raises(ValueError, match="lattices"):
        m.lj_md_cg_attach(fake_handle, 10, lats, _t((3, 50), torch.int64), _t((3, 5), torch.float64), stream=0)


def test_energy_takes_its_shape_from_the_handle():
    import inspect

    import paper_2101_01160_amd as m
    assert list(inspect.signature(m.lj_md_energy).parameters) == ["h", "stream"]
