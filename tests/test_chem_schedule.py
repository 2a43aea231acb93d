"""The chemistry schedule of the porous-electrode benchmark (one backward-Euler
sub-step with two Newton iterations per lattice step) against a converged one.

The chemistry stage integrates the gas and surface balances over the lattice step
with fixed sub-steps and Newton iterations (reading R13).  On a C3 sub-grid (the
same gas, porosity recipe and 20-reaction mechanism), from the initial state and
from the state after 20 steps, the species source and the coverage change of the
1 x 2 schedule are within 2e-5 (normwise, relative) of a 16 sub-step x 8 iteration
reference, and those of the 4 x 6 default within 5e-6: the difference is the
first-order time error of backward Euler (4 sub-steps cut it about 5x), not an
unconverged Newton solve."""
from dataclasses import replace

import numpy as np
import pytest

from oracle.lbm_oracle import Oracle
from workloads import synth


@pytest.mark.parametrize("steps", [0, 20])
def test_benchmark_chemistry_schedule_is_within_2e5_of_converged(steps):
    w = synth.config3(nx=8, ny=6, nz=4)
    assert (w.mech.n_sub, w.mech.n_newton) == (1, 2)
    o = Oracle(w)
    o.step(steps)
    mac = o.macro()
    th0 = o.theta.copy()
    out = {}
    for sched in ((1, 2), (4, 6), (16, 8)):
        o.mech = replace(w.mech, n_sub=sched[0], n_newton=sched[1])
        out[sched] = o.chemistry(mac)
    ref_src, ref_th = out[(16, 8)]
    for sched, bound in (((1, 2), 2e-5), ((4, 6), 5e-6)):
        src, th = out[sched]
        e_src = np.abs(src - ref_src).max() / np.abs(ref_src).max()
        e_th = np.abs(th - ref_th).max() / np.abs(ref_th - th0).max()
        assert e_src < bound and e_th < bound, (sched, e_src, e_th)
