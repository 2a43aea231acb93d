"""lbm_get_diagnostics_static (the entry point that allocates nothing, its scratch a
file-scope device array) against lbm_get_diagnostics, bit for bit, on two calls in a
row: a C3 sub-grid with chemistry, then a smaller D2Q9 lattice (the second call finds
the first call's partials in the array and must not be affected by them); and the
size limit is refused with LBM_EINVAL, not run."""
import numpy as np
import pytest

from workloads import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available()
    from paper_2409_02930_amd import lbm as _lbm
    return _lbm


def _same(a, b):
    for k in ("species_mass", "mixture_mass", "mixture_momentum", "energy_total", "min_population",
              "n_nonfinite", "steps_done", "rc"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (k, a[k], b[k])


def test_static_diagnostics_equal_the_allocating_ones_on_two_calls(lbm):
    big = synth.config3(nx=48, ny=24, nz=16)          # 18432 nodes, 6 lattices, chemistry
    small = synth.config1(nx=20, ny=12)               # 240 nodes, 3 lattices
    for w, steps in ((big, 3), (small, 5)):
        lat = lbm.lattice_from_workload(w)
        lat.step(steps)
        ref = lat.diagnostics()
        got = lat.diagnostics_static()
        print(w.name, w.N, "nodes:", got, flush=True)
        _same(got, ref)
        got2 = lat.diagnostics_static()               # the array now holds this call's contents
        _same(got2, ref)
        lat.close()


def test_static_diagnostics_refuse_a_lattice_beyond_the_scratch(lbm):
    w = synth.config1(nx=4096, ny=4096)              # 65536 blocks x 7 doubles > 2^18
    lat = lbm.lattice_from_workload(w)
    d = lat.diagnostics_static(check=False)
    lat.close()
    assert d["rc"] == lbm.LBM_EINVAL
