"""CPU oracle for the generalized-harmonic (GH) shell evolution.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (the HIP library and its Python binding) never imports it, and this
package never imports the product.

What it is: a plain, slow, FP64 (or complex128, for complex-step derivatives)
NumPy implementation of what the GPU path computes, written step by step from
the paper (Lewis & Pfeiffer, arXiv:1804.09101) where the paper speaks, and from
the published first-order GH formulation (Lindblom, Scheel, Kidder, Owen & Rinne
2006) where it does not.  Derivatives are taken by spectral *transforms*
(PhysToSpec, coefficient-space derivative, SpecToPhys; the paper's
Spectral Operations section, eqs. SpecToPhys / PhysToSpec / Deriv), never by the
dense traced matrices the GPU path uses.

Modules:
  grid      collocation points and quadrature weights on a shell I1 x S2
  spectral  Chebyshev and real Y_lm transforms, derivatives, angular filter
  gh        pointwise GH algebra: RHS, constraints, characteristic fields
  domain    a stack of shells: Cartesian gradient, boundary treatment,
            SSP-RK3 step, filter, constraint norm
  tensor_filter  the tensor-coupled angular filter (total angular momentum)
  dp5       Dormand-Prince 5(4) tableau and step control
  kerr_schild  the oracle's own exact Kerr-Schild spacetimes (hyper-dual
            derivatives), used by its pins instead of the input generator

All functions accept complex128 inputs so that complex-step differentiation
gives exact directional derivatives (used as the reference gradient).
"""

from . import grid, spectral, gh, domain, tensor_filter, kerr_schild  # noqa: F401
