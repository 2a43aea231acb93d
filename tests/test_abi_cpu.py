"""The C-ABI library loads and exports every entry point include/lbm.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "lbm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for core in ("lbm_init", "lbm_set_porous_field", "lbm_set_mechanism", "lbm_step", "lbm_moments"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2409_02930_amd import lbm
    lib = ctypes.CDLL(lbm.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(lbm.EXPORTED) == _declared()


def test_binding_rejects_bad_config_without_gpu_compute():
    """Validation happens on the host before any device call."""
    import numpy as np
    from paper_2409_02930_amd import lbm
    with pytest.raises(lbm.LBMError) as e:
        lbm.Lattice(2, 4, 4, 1, [0.002, 0.028], np.full((2, 2), 0.2), np.full((2, 16), 0.7),
                    np.full(16, 1073.0))
    assert e.value.code == lbm.LBM_EINVAL


def _cfg_args():
    import numpy as np
    M, N = 2, 16
    return dict(dim=2, nx=4, ny=4, nz=1, molar_mass=[0.002, 0.028], D_ref_lat=np.full((M, M), 0.2),
                X0=np.full((M, N), 0.5), T0=np.full(N, 1073.0))


@pytest.mark.parametrize("bad", ["precision", "species", "asymmetric_D", "extents", "periodic_one_side",
                                 "inlet_without_X", "energy_without_thermo", "theta_ref"])
def test_config_validation_on_host(bad):
    """Every rejected configuration fails with LBM_EINVAL before any device work."""
    import numpy as np
    from paper_2409_02930_amd import lbm
    a = _cfg_args()
    kw = {}
    if bad == "precision":
        kw["precision"] = 2
    elif bad == "species":
        a["molar_mass"] = [0.002] * 6
        a["D_ref_lat"] = np.full((6, 6), 0.2)
        a["X0"] = np.full((6, 16), 1.0 / 6)
    elif bad == "asymmetric_D":
        a["D_ref_lat"] = np.array([[0.2, 0.2], [0.3, 0.2]])
    elif bad == "extents":
        a["nz"] = 2
    elif bad == "periodic_one_side":
        kw["bc_lo"], kw["bc_hi"] = lbm.BC_PERIODIC, lbm.BC_BOUNCEBACK
    elif bad == "inlet_without_X":
        kw["bc_lo"], kw["bc_hi"] = lbm.BC_INLET, lbm.BC_OUTFLOW
    elif bad == "energy_without_thermo":
        kw["energy_on"] = True
    elif bad == "theta_ref":
        kw["theta_ref"] = 1.5
    with pytest.raises(lbm.LBMError) as e:
        lbm.Lattice(a["dim"], a["nx"], a["ny"], a["nz"], a["molar_mass"], a["D_ref_lat"], a["X0"], a["T0"], **kw)
    assert e.value.code == lbm.LBM_EINVAL, str(e.value)
