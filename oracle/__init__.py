"""Plain, slow FP64 CPU oracle of the spectral point-mass filter.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or calls this package; only ``tests/``, the smoke
check and the CPU-baseline leg of the benchmark do.  It shares no code with the
GPU path: its inputs come from ``workloads`` (seeded generators only).

Every routine follows a definition of the paper written out directly:

* DFT of eq. fourtrsf (Sec. IV) as a dense matrix, no FFT;
* the minimal-oscillation trigonometric interpolant of eq. interFreq and its first
  and second derivatives (eq. secDer), as dense matrices;
* the moving-grid Fokker-Planck equation of Sec. II.B (eqs. movFPEadv, easyFPE),
  integrated in physical grid space by classic RK4 (method of lines), or by the
  implicit Euler step of Sec. V.A, or exactly (a per-mode exponential), or by
  the explicit finite-difference baseline of eq. FDM (step matrices of eq. fdiff),
  or a sine-series variant of the spectral update (exact zero boundary values);
* Chebyshev differentiation (Sec. IV.B) on Chebyshev-Gauss-Lobatto nodes;
* the Bayes rule of Sec. I.A (eq. filt) applied point by point, with the
  normalisation of Sec. III.A (eq. PDF_pm).

Where the paper is silent or inconsistent the oracle takes the readings listed
in the design notes (trace sign, Euler sign, Nyquist handling, grid design,
re-interpolation kernel, substep clamp).
"""
from .pmf import (State, create, predict, update, moments, design_grid, nodes,
                  quadrature_weights, interpolate, substeps, loglik_field,
                  boundary_fraction)

__all__ = ["State", "create", "predict", "update", "moments", "design_grid", "nodes",
           "quadrature_weights", "interpolate", "substeps", "loglik_field",
           "boundary_fraction"]
