"""Oracle: plain, slow, obviously correct CPU implementation of the shell-binning and
Born-convergence path, used ONLY as test infrastructure.

Only tests/, the smoke check and the bench's CPU-baseline leg import this
package.  It shares no code with the HIP library (paper_1801_05745_amd) and
never imports it.

  healpix    exact RING ang2pix / pix2ang and an independent projection brute force
  binning    FP64 C particle loop with guard bands + exact resolution of flagged instances
  cosmology  D(z), lensing weights (delta and Smail n(z) sources), nbar, kappa, adjoint
  spectra    spherical-harmonic coefficients, C_l and their covariance over realisations
"""

from . import binning, cosmology, healpix, spectra  # noqa: F401
