"""The oracle's complex-step tangent (tests/oracle_tangent.py) against central finite
differences of the oracle itself: the directional derivative of the outlet-flux
objective along a random porosity direction and along the pore radius, on the C5
physics (inlet / outflow, GRF porosity, Knudsen drag) for 20 steps.  The finite
differences carry their own truncation and cancellation error of about 1e-9; the
tangent must agree with them to that level."""
from dataclasses import replace

import numpy as np

from oracle.lbm_oracle import Oracle
from oracle_tangent import outlet_flux_tangent
from workloads import synth


def test_complex_step_tangent_matches_central_differences():
    w = synth.config5(nx=24, ny=8)
    T = 20
    v = np.random.default_rng(0).standard_normal(w.N)
    J, dJ = outlet_flux_tangent(w, T, 0, dphi=v)
    assert abs(J - Oracle(w).outlet_flux(T, 0)) <= 1e-13 * abs(J)      # the real part is the run itself
    h = 1e-6
    fd = (Oracle(replace(w, phi=w.phi + h * v)).outlet_flux(T, 0)
          - Oracle(replace(w, phi=w.phi - h * v)).outlet_flux(T, 0)) / (2 * h)
    assert abs(fd / dJ - 1.0) < 1e-8, (fd, dJ)
    _, dr = outlet_flux_tangent(w, T, 0, drp=1.0)
    hr = 1e-6 * w.pore_radius
    fdr = (Oracle(replace(w, pore_radius=w.pore_radius + hr)).outlet_flux(T, 0)
           - Oracle(replace(w, pore_radius=w.pore_radius - hr)).outlet_flux(T, 0)) / (2 * hr)
    assert abs(fdr / dr - 1.0) < 1e-8, (fdr, dr)
