"""Direct solvers of the discrete cylindrical Poisson problem (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The method of Sec. 3 is exact (up to rounding): its result is the unique
solution of the undecomposed 3-D system ``A u = s rho + b^D`` on the interior
nodes (Eqs. (mode_rhs), (full_finite_volume_row)), with boundary nodes at
their Dirichlet values.  ``solve_dense`` and ``solve_sparse`` compute exactly
that definition.  ``solve_separable`` is a second exact direct method for
grids too large for sparse LU: FFT in theta, sine transform in z, tridiagonal
solve in r (the classical fast Poisson solver; it needs uniform z, which this
grid has).  ``solve_mode`` solves one 2-D system ``(A_0 + lambda M) u = b`` of
Eq. (shifted_operator_family); ``solve_modes`` is the whole method of Sec. 3
with a direct solve per mode, for meshes of any spacing.
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fv, spectral
from .spectral import discrete_eigenvalue


def _problem_rhs(grid, rho, bc=None, phi_boundary=None):
    if phi_boundary is None:
        phi_boundary = fv.boundary_values(grid, bc)
    return fv.rhs(grid, rho, phi_boundary), phi_boundary


def solve_dense(grid: fv.Grid, rho, bc=None, phi_boundary=None) -> np.ndarray:
    """Dense LU (``numpy.linalg.solve``) of the 3-D system; tiny grids only."""
    b, pb = _problem_rhs(grid, rho, bc, phi_boundary)
    A = fv.assemble(grid).toarray()
    u = np.linalg.solve(A, b.ravel())
    return fv.with_boundary(grid, u, pb)


def solve_sparse(grid: fv.Grid, rho, bc=None, phi_boundary=None) -> np.ndarray:
    """Sparse direct solve (SuperLU, minimum-degree ordering on A^T + A) of the 3-D system."""
    b, pb = _problem_rhs(grid, rho, bc, phi_boundary)
    A = fv.assemble(grid).tocsc()
    lu = spla.splu(A, permc_spec="MMD_AT_PLUS_A", options={"SymmetricMode": True})
    u = lu.solve(b.ravel())
    return fv.with_boundary(grid, u, pb)


def mode_operator(A0: sp.spmatrix, mu: np.ndarray, lam: float) -> sp.csr_matrix:
    """``A_m = A_0 + lambda_m M`` with ``M = diag(mu)``, Eq. (shifted_operator_family)."""
    return (sp.csr_matrix(A0) + lam * sp.diags(np.ravel(mu))).tocsr()


def plane_matrix(grid: fv.Grid) -> sp.csr_matrix:
    """The 2-D radial-axial operator A_0 on one plane's interior nodes (row index k*(nr-2)+i)."""
    nz, nr = grid.nz - 2, grid.nr - 2
    K, I = np.meshgrid(np.arange(nz), np.arange(nr), indexing="ij")
    row = K * nr + I
    rows, cols, vals = [row.ravel()], [row.ravel()], [grid.D0.ravel()]
    for mask, col, g in (
        (I > 0, row - 1, grid.G_rm),
        (I < nr - 1, row + 1, grid.G_rp),
        (K > 0, row - nr, grid.G_zm),
        (K < nz - 1, row + nr, grid.G_zp),
    ):
        rows.append(row[mask])
        cols.append(col[mask])
        vals.append(-g[mask])
    n = nz * nr
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()


def solve_mode(grid: fv.Grid, lam: float, b_plane: np.ndarray) -> np.ndarray:
    """Solve the 2-D mode system ``(A_0 + lambda M) u = b`` (interior nodes of one plane)."""
    A = mode_operator(plane_matrix(grid), grid.mu, lam).tocsc()
    return spla.spsolve(A, np.ravel(b_plane)).reshape(grid.nz - 2, grid.nr - 2)


def solve_modes(grid: fv.Grid, rho, bc=None, phi_boundary=None) -> np.ndarray:
    """The method of Sec. 3 with exact mode solves: the right-hand side's
    azimuthal DFT (Eq. (azimuthal_dft)), a sparse direct solve of
    ``A_0 + lambda_m M`` on every real plane (Eqs. (shifted_operator_family),
    (mode_rhs)), and the inverse DFT.  Exact up to rounding on any mesh; the
    cosine and sine planes of one mode share a factorisation."""
    b, pb = _problem_rhs(grid, rho, bc, phi_boundary)
    planes = spectral.forward(np.reshape(b, grid.interior_shape))
    lam = spectral.plane_eigenvalues(grid.ntheta, float(grid.dtheta))
    A0 = plane_matrix(grid)
    out = np.empty_like(planes)
    factors = {}
    for p in range(grid.ntheta):
        key = float(lam[p])
        if key not in factors:
            factors[key] = spla.splu(mode_operator(A0, grid.mu, key).tocsc())
        out[p] = factors[key].solve(planes[p].ravel()).reshape(planes[p].shape)
    return fv.with_boundary(grid, spectral.inverse(out).ravel(), pb)


def solve_separable(grid: fv.Grid, rho, bc=None, phi_boundary=None, workers=None) -> np.ndarray:
    """Exact direct solve by FFT in theta, DST-I in z and a tridiagonal solve in r.

    With uniform z spacing the axial conductances of node i do not depend on k
    (``G_{z,-} = G_{z,+} = r_i dr / dz``), so the axial three-point operator is
    ``G_z(i)`` times the Dirichlet second difference, diagonalised by the
    type-I sine transform with eigenvalues ``4 sin^2(pi p / (2 (Nz - 1)))``.
    The azimuthal part is ``mu_i lambda_m`` (Eq. (discrete_azimuthal_eigenvalue)).
    What remains for each (m, p) is a symmetric tridiagonal system in r,
    solved with ``scipy.linalg.solve_banded``-equivalent Thomas elimination
    vectorised over all (m, p).  Runs in ``grid.dtype``: an extended-precision
    grid (``numpy.longdouble``, scipy's transforms keep it) gives the exact
    discrete solution of an FP64 ``rho`` far below the FP64 rounding floor.
    """
    if not getattr(grid, "uniform", True):
        raise ValueError("the separable solver needs the uniform vertex-centred grid")
    b, pb = _problem_rhs(grid, rho, bc, phi_boundary)
    nt, nz, nr = grid.interior_shape
    gz = grid.G_zm[0]
    if not (np.array_equal(grid.G_zm, np.broadcast_to(gz, grid.G_zm.shape))
            and np.array_equal(grid.G_zm, grid.G_zp)):
        raise ValueError("separable solve needs k-independent axial conductances")
    t = grid.dtype
    bh = scipy.fft.rfft(b, axis=0, workers=workers)  # (nm, nz, nr) complex
    bh = scipy.fft.dst(bh, type=1, axis=1, workers=workers)
    nm = bh.shape[0]
    lam = discrete_eigenvalue(np.arange(nm), nt, grid.dtheta, dtype=t)  # (nm,)
    p = np.arange(1, nz + 1, dtype=t)
    pi = t(2) * np.arccos(t(0))
    sig = t(4) * np.sin(pi * p / (t(2) * t(nz + 1))) ** 2  # (nz,)
    gw = grid.G_rm[0]  # (nr,)
    ge = grid.G_rp[0]
    mu = grid.mu[0]
    diag = (gw + ge)[None, None, :] + gz[None, None, :] * sig[None, :, None] + mu[None, None, :] * lam[:, None, None]
    # Thomas elimination along r: sub-diagonal -gw[i] (to i-1), super-diagonal -ge[i] (to i+1)
    cp = np.empty(diag.shape, dtype=diag.dtype)
    dp = np.empty(bh.shape, dtype=bh.dtype)
    cp[..., 0] = -ge[0] / diag[..., 0]
    dp[..., 0] = bh[..., 0] / diag[..., 0]
    for i in range(1, nr):
        den = diag[..., i] + gw[i] * cp[..., i - 1]
        cp[..., i] = -ge[i] / den
        dp[..., i] = (bh[..., i] + gw[i] * dp[..., i - 1]) / den
    uh = np.empty_like(dp)
    uh[..., nr - 1] = dp[..., nr - 1]
    for i in range(nr - 2, -1, -1):
        uh[..., i] = dp[..., i] - cp[..., i] * uh[..., i + 1]
    uh = scipy.fft.idst(uh, type=1, axis=1, workers=workers)
    u = scipy.fft.irfft(uh, n=nt, axis=0, workers=workers)
    return fv.with_boundary(grid, u, pb)


def residual_norm(grid: fv.Grid, phi, rho, bc=None, phi_boundary=None) -> float:
    """Relative residual ``||s rho - A_full phi||_2 / ||s rho + b^D||_2`` in ``grid.dtype``.

    ``A_full phi = s rho`` at every interior node is the cell balance
    Eq. (full_finite_volume_row) with the boundary terms kept on the left;
    boundary nodes of ``phi`` are replaced by the prescribed values first.
    """
    b, pb = _problem_rhs(grid, rho, bc, phi_boundary)
    full = np.array(pb, dtype=grid.dtype, copy=True)
    full[:, 1:-1, 1:-1] = np.asarray(phi, dtype=grid.dtype)[:, 1:-1, 1:-1]
    s_rho = grid.s_eps0 * np.asarray(rho, dtype=grid.dtype)[:, 1:-1, 1:-1] / grid.dtype(fv.EPS0)
    r = s_rho - fv.apply_full(grid, full)
    return float(np.sqrt(np.sum(r * r)) / np.sqrt(np.sum(b * b)))
