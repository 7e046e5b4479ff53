"""CPU checks of the Python binding's host logic: an object that holds raw
device pointers, or a handle that uses another one, keeps what it points
into alive (a temporary passed in would otherwise be freed, and its memory
handed to the next allocation of that size, before the library reads it)."""
import gc
import weakref

import pytest


def _agc():
    try:
        from paper_2605_04773_amd import agc
    except (ImportError, OSError) as e:
        pytest.skip(f"libagc.so not loadable here: {e}")
    return agc


class _Ctx:
    device = None
    h = None


class _Mesh:
    h = None
    n_verts = 4
    n_elems = 1
    ctx = _Ctx()


def test_problem_keeps_its_tensors(monkeypatch):
    import torch
    agc = _agc()
    monkeypatch.setattr(agc, "_dev", lambda t, *a, **k: t)   # the device checks need a GPU
    tensors = [torch.zeros(4, 2, dtype=torch.int32), torch.zeros(4, dtype=torch.uint8),
               torch.zeros(1, 144, dtype=torch.float64), torch.zeros(4, 3, dtype=torch.float64),
               torch.zeros(4, 3, dtype=torch.float64)]
    refs = [weakref.ref(t) for t in tensors]
    ptrs = [t.data_ptr() for t in tensors]
    prob = agc.make_problem(_Mesh(), *tensors)
    del tensors
    gc.collect()
    assert all(r() is not None for r in refs)
    assert [prob.edges, prob.tags, prob.elem_H, prob.g, prob.rest] == ptrs
    del prob
    gc.collect()
    assert all(r() is None for r in refs)


def test_newton_handle_keeps_its_mesh():
    agc = _agc()
    mesh = _Mesh()
    ref = weakref.ref(mesh)
    nw = agc.Newton(_Ctx(), None, 4, 1, mesh)
    del mesh
    gc.collect()
    assert ref() is not None and nw.mesh is ref()
