"""CPU checks of the Python binding's argument marshalling: every device vector
handed to the library must have exactly the length the call reads and writes,
and per-problem pointer lists must have one entry per problem.  A wrong length
raises ValueError before the library (or the GPU) is touched.  The C ABI's own
argument checks (null context, bad checkpoint fields) are reached without a GPU
as well."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2412_20205_amd import igamg


class _FakeSolver(igamg.Solver):
    """A Solver whose sizes come from a table instead of a context."""

    def __init__(self, sizes, degree=3, geometry=igamg.QUARTER_ANNULUS):
        self._h = None
        self._sizes = list(sizes)  # level 0 .. L
        self.geometry, self.n_el, self.degree = geometry, 0, degree

    @property
    def ndof(self):
        return self._sizes[-1]

    @property
    def num_levels(self):
        return len(self._sizes)

    def level_ndof(self, level):
        return self._sizes[level]

    def close(self):
        self._h = None


SIZES = [25, 81, 289]


def _v(n, dtype=torch.float64):
    return torch.zeros(n, dtype=dtype)


def _raises_length(fn):
    with pytest.raises(ValueError, match="entries"):
        fn()


def _raises_device(fn):
    # right length: the next check (device tensor) fails, still before any call
    with pytest.raises(ValueError, match="device tensor"):
        fn()


def test_finest_level_vectors_checked():
    s = _FakeSolver(SIZES)
    n = SIZES[-1]
    for call in (lambda x: s.vcycle(x), lambda x: s.residual(x), lambda x: s.solve(x),
                 lambda x: s.solve_fgmres(x), lambda x: s.get_rhs(x), lambda x: s.set_rhs(x),
                 lambda x: s.get_state(x)):
        _raises_length(lambda: call(_v(n - 1)))
        _raises_length(lambda: call(_v(n + 1)))
        _raises_device(lambda: call(_v(n)))


def test_set_rhs_host_array_checked():
    s = _FakeSolver(SIZES)
    with pytest.raises(ValueError):
        s.set_rhs(np.zeros(SIZES[-1] - 1))


def test_iterate_blocks_checked():
    s = _FakeSolver(SIZES)
    n = SIZES[-1]
    q = 5
    _raises_length(lambda: s.extrapolate(igamg.RRE, q, _v(n), iterates=_v((q + 1) * n)))
    _raises_length(lambda: s.extrap_coeffs(igamg.RRE, q, _v((q + 2) * n - 1)))
    _raises_device(lambda: s.extrap_coeffs(igamg.RRE, q, _v((q + 2) * n)))


def test_level_vectors_checked():
    s = _FakeSolver(SIZES)
    for l in (1, 2):
        n, nc = SIZES[l], SIZES[l - 1]
        _raises_length(lambda: s.apply(l, _v(n), _v(nc)))
        _raises_length(lambda: s.smooth(l, _v(nc), _v(n)))
        _raises_length(lambda: s.restrict(l, _v(n), _v(n)))
        _raises_length(lambda: s.prolong_add(l, _v(n), _v(n)))
        _raises_device(lambda: s.restrict(l, _v(n), _v(nc)))
        _raises_device(lambda: s.prolong_add(l, _v(nc), _v(n)))
        _raises_length(lambda: s.smoother_forward(l, _v(n, torch.float32), _v(n + 1, torch.float32)))
        _raises_length(lambda: s.smoother_loss_grad(l, _v(nc, torch.float32), _v(n, torch.float32)))
    _raises_length(lambda: s.coarse_solve(_v(SIZES[0]), _v(SIZES[1])))


def test_mode_table_shape_checked():
    s = _FakeSolver(SIZES)
    with pytest.raises(ValueError, match="shape"):
        s.set_rhs_field(np.zeros((64, 5)))
    with pytest.raises(ValueError, match="shape"):
        s.set_rhs_field(np.zeros(256))
    cube = _FakeSolver(SIZES, geometry=igamg.UNIT_CUBE)
    with pytest.raises(ValueError, match="shape"):
        cube.set_rhs_field(np.zeros((8, 4)))


def test_batch_pointer_list_checked():
    b = object.__new__(igamg.Batch)
    b._h = None
    b.instances = [_FakeSolver([9, 49]), _FakeSolver([16, 100])]
    b.problems = [None, None]
    with pytest.raises(ValueError, match="problems"):
        b.solve([_v(49)])
    with pytest.raises(ValueError, match="problems"):
        b.solve([_v(49), _v(100), _v(100)])
    _raises_length(lambda: b.solve([_v(49), _v(99)]))
    _raises_device(lambda: b.solve([_v(49), _v(100)]))


class _FakeSet(igamg.Set1D):
    def __init__(self, sizes):
        self._h = None
        self._sizes = sizes
        self.problems = [{} for _ in sizes]

    def ndof(self, i):
        return self._sizes[i]

    def close(self):
        self._h = None


def test_set1d_vectors_checked():
    s = _FakeSet([65, 130])
    with pytest.raises(ValueError, match="problems"):
        s.solve([_v(65)])
    with pytest.raises(ValueError, match="problems"):
        s.cycles([_v(65), _v(130), _v(1)])
    _raises_length(lambda: s.solve([_v(65), _v(129)]))
    _raises_length(lambda: s.set_rhs(1, _v(65)))
    _raises_length(lambda: s.get_rhs(0, _v(130)))


def test_state_calls_reject_null_context_and_bad_fields():
    L = igamg.lib()
    st = igamg.State()
    assert L.igamg_get_state(None, None, ctypes.byref(st)) == igamg.EINVAL
    assert L.igamg_set_state(None, ctypes.byref(st)) == igamg.EINVAL
    assert L.igamg_set_state(None, None) == igamg.EINVAL
