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
