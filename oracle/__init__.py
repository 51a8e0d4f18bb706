"""Oracle: a plain, slow FP64 CPU implementation of the RadioLensfit hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute this package; only the test suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path
(no kernels, headers, helpers or tables) and never takes an input or an
expected value produced by the HIP path.

Every function follows a passage of Rivi & Miller, "RadioLensfit: an HPC
tool for accurate galaxy shape measurement with SKA" (arXiv 2203.14071):

  model.py       Eq. 1-3 (exponential-disk visibility, shear matrix), Eq. 4
                 (scale-flux relation), the sky model of Sec. 2.2
  extract.py     Sec. 2.3: neighbour subtraction, phase shift, facet sizing
                 and averaging into a coarse uv grid
  likelihood.py  Sec. 2.4: chi-squared likelihood on the facet, analytic flux
                 marginalisation, numerical scale-length marginalisation with
                 a log-normal prior
  estimate.py    Sec. 2.4 and 4.1: mean and standard deviation of the
                 ellipticity samples above 5 % of the maximum likelihood,
                 the variance test for bad fits
  position.py    Sec. 2.4: marginalisation over the source position with a
                 uniform prior through the cross-correlation of the facet
                 data with the model (reading in its docstring)
  sequential.py  Sec. 2.1, 2.4, 3.1: chunked sequential sky-model refinement
                 and the refit of bad fits
  refine.py      Sec. 2.4: adaptive refinement of the sampled likelihood
                 around its maximum (nested grids)
  mlp.py         the learned grid-narrowing network (not in the paper): an
                 FP64 forward/backward used to check the BF16 kernels

Where the paper is silent or ambiguous the reading taken is stated in the
docstring of the function concerned.  All arithmetic is FP64 with the host
libm (through numpy); there is no blocking, fusion or reordering beyond the
definitions.
"""
from .model import (ARCSEC, C_LIGHT, wavelengths, spectral_factor, n_minus_one,
                    shape_inv_t, disk_vis, sky_model, alpha_from_flux)
from .extract import Facet, facet_theta, extract_facet, extract_facets
from .likelihood import (alpha_knots, spline_quadrature_weights, log_normal_prior,
                         e_grid, loglike_alpha, marginal_surface, log_alpha_weights)
from .estimate import Estimate, estimate, FLAG_BAD_VAR, FLAG_EMPTY, FLAG_EDGE, FLAG_FALLBACK
from .fit import (Params, fit_source, fit_sources, narrowed_fit, window_rejected, lattice_window,
                  lattice_narrowed_fit)
from .sequential import FLAG_REFIT, SkyCatalogue, fit_sequential
from .refine import FLAG_REFINED, refine_source
from .position import offset_grid, loglike_alpha_offsets, marginal_surface_pos, fit_source_pos
