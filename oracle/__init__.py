"""CPU oracle for the full-spectrum cylindrical Poisson solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute this package; only the test-suite, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the GPU library.

What it computes (plain FP64, or extended precision where stated):

* ``fv``        -- the finite-volume coefficients of App. A (face conductances,
                   shift coefficient, charge scale), the undecomposed 3-D
                   seven-point operator of Sec. 3.1 on the vertex-centred annular
                   grid, its right-hand side (charge term plus Dirichlet terms),
                   and the operator applied to a full potential.
* ``spectral``  -- the azimuthal DFT of Eq. (azimuthal_dft) written out as sums,
                   split into real "planes", its inverse, and the exact discrete
                   eigenvalue of Eq. (discrete_azimuthal_eigenvalue).
* ``nn``        -- the learned preconditioner's three-layer 3x3 convolution
                   network: forward, loss, back-propagated gradients and an
                   Adam step in FP64, optionally with the GPU's BF16 operand
                   rounding (the brief fixes the network; the paper has none).
* ``solvers``   -- the plain definition: a direct solve of the undecomposed 3-D
                   system (dense for tiny grids, sparse LU otherwise), the 2-D
                   shifted mode system of Eq. (shifted_operator_family), and an
                   exact separable (FFT / sine-transform / tridiagonal) direct
                   solver for grids too large for sparse LU.

Every function names the passage it follows.  Each is pinned by the
``-m "not gpu"`` tests against values the paper prints, closed forms,
brute force or library routines; no function here is "parity unpinned".
"""
from . import fv, nn, spectral, solvers  # noqa: F401
from .fv import EPS0  # noqa: F401
