"""Complex-step tangent of the oracle's outlet-flux objective (test infrastructure).

J(phi + i h v, r_p + i h s) = J + i h (dJ/dphi . v + dJ/dr_p s) + O(h^2), so the
imaginary part over h is the directional derivative to rounding, with no
cancellation (h = 1e-30).  The oracle's arithmetic is analytic in phi and r_p on
the isothermal, reaction-free path the adjoint covers (its branches compare real
parts only), so running it on complex inputs gives the exact tangent.  Tortuosity
is held fixed, as in the adjoint.
"""
from dataclasses import replace

import numpy as np

from oracle.lbm_oracle import Oracle

H = 1e-30


def outlet_flux_tangent(w, steps, species=0, dphi=None, drp=0.0):
    """(J, dJ along (dphi, drp)) from one complex run of the oracle."""
    o = Oracle(w)
    if dphi is not None:
        o.phi = o.phi + 1j * H * np.asarray(dphi, dtype=np.float64)
    if drp:
        o.w = replace(o.w, pore_radius=w.pore_radius + 1j * H * drp)
    o._init_state()
    o.fa = o.fa.astype(np.complex128)          # every state array complex from the start
    o.f = o.f.astype(np.complex128)
    J = o.outlet_flux(steps, species)
    return float(np.real(J)), float(np.imag(J)) / H
