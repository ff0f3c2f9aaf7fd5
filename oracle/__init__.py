"""FP64 CPU oracle of the joint SOS/image reconstruction's forward model.

TEST INFRASTRUCTURE ONLY.  Nothing in the reconstruction library imports,
links or runs this package; only the tests, the smoke check and the
measuring legs of the benchmark (its CPU baselines and its precision
report) do, and none of them feeds a kernel.  It shares no code with the HIP path:
it computes its own geometry, its own grids and its own sums, in float64
(numpy for the delay-and-sum stack, torch float64 on the CPU elsewhere so
that the gradient of the loss is obtained by reverse-mode differentiation,
as the paper does).

Every function restates one passage of Li, Cui, Ma, Alexander,
"Coordinate-based Speed of Sound Recovery for Aberration-Corrected
Photoacoustic Computed Tomography" (ICCV 2025):

  das.py      Eq. DAS                  delay-and-sum image per extra delay
  patches.py  Sec. 3.3 / Supp. S1.4    Gaussian-windowed patches and their FFT
  sos.py      Sec. 3.3                 interpolated pixel-grid SOS with fixed background
  rays.py     Eq. TOF, Eq. wf          straight-ray wavefront error per element
  psf.py      Eq. TF                   transfer function / PSF from the wavefront
  deconv.py   Eq. fm_fourier, Eq. multi-deconv   pseudo-inverse deconvolution
  loss.py     Eq. jr                   |k|-weighted residual + TV, and its gradient
  adam.py     Sec. 3.3 (Adam)          the optimiser step
  stitch.py   Supp. S1.4               Gaussian-weighted patch stitching

Readings where the paper is silent or ambiguous (conjugate transpose in the
pseudo-inverse, FFT sign convention, interpolation of the wavefront between
elements, midpoint ray quadrature, Tikhonov eps, TV form) are stated in the
docstrings of the functions that take them.
"""
from . import geometry, das, patches, sos, rays, psf, deconv, loss, adam, stitch  # noqa: F401
