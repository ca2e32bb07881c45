"""MI355X (gfx950) implementation of the scheme-III gradient path of
Bharadwaj, Mulder & Drijkoningen, "A parameterization analysis for acoustic
full-waveform inversion of sub-wavelength anomalies" (arXiv:1804.01184):
2-D variable-density acoustic staggered-grid modelling, the least-squares
misfit and its adjoint-state gradient with respect to (K, rho), chain-ruled
to the parameterizations of Table 1.

Past that path: steepest descent (``inversion``), error bowls (``bowls``),
diffraction patterns (``patterns``), and schemes I and II, Born modelling
in the frequency domain (``born``).

The computation lives in the HIP library ``libfwi2d.so`` (C ABI in
``include/fwi2d.h``); ``api`` binds it to torch device memory and streams.
"""
from . import workloads  # noqa: F401  (input generators; no GPU needed)

__all__ = ["workloads"]
