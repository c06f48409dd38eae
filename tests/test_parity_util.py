"""The phi-shift form of the rounding scale used by the largest-degree parity
test equals the fully traced one (the angular operators commute with shifts
of the uniform phi grid)."""

import numpy as np

from oracle import domain
from paper_1804_09101_amd import configs
from parity_util import rounding_scale, rounding_scale_by_shifts, _abs_operator_by_shifts, _traced


def test_shift_form_equals_full_trace():
    shells = [(0, 5, 7, 1.8, 2.6), (0, 4, 7, 2.6, 3.5)]
    d = domain.Domain([domain.Shell(*s) for s in shells])
    wl = configs.Workload("x", shells, [(1.0, 0.3, (0.2, 0.3, 0.4))], [configs.GAMMA_DEFAULT], [1e-3], None, 1, None)
    u0, _, _, _ = wl.initial_data(d.xyz(), d.offsets)
    u0 = u0 + 1e-2 * np.random.default_rng(0).standard_normal(u0.shape)
    sph = d.spheres[7]
    for fn in (sph.d_dtheta, sph.d_dphi):
        full = np.abs(_traced(lambda v: fn(v.reshape(sph.nth, sph.nph)).ravel(), sph.S))   # [output, input]
        by_shifts = _abs_operator_by_shifts(fn, sph.nth, sph.nph)                          # [input, output]
        assert np.max(np.abs(full.T - by_shifts)) < 1e-12 * np.max(full)
    for j, b in enumerate(d.split(u0, 50)):
        a, c = rounding_scale(d, j, b), rounding_scale_by_shifts(d, j, b)
        assert abs(a - c) < 1e-12 * a
