"""Pins of the oracle's general-geometry grids (CPU only): the cell-centred
finite volumes of App. A with half-cell Dirichlet faces, and vertex-centred
grids on non-uniform points."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import fv, solvers, spectral

stretched = W.stretched_points

EPS0 = fv.EPS0


def test_half_cell_dirichlet_example(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "appendix_a_dirichlet_cell.json")))
    c, e = g["cell"], g["expected"]
    # one interior cell: west point at distance 1, the Dirichlet face half a cell east
    grid = fv.Grid.general(r=[1.0, 2.0, 2.5], z=[-1.0, 0.0, 1.0], r_lo=[c["r_face_lo"]],
                           r_hi=[c["r_face_hi"]], z_lo=[-0.5], z_hi=[0.5], ntheta=1)
    assert grid.G_rm[0, 0] == pytest.approx(e["G_r_minus"], rel=1e-15)
    assert grid.G_rp[0, 0] == pytest.approx(e["G_r_plus_dirichlet"], rel=1e-15)
    assert grid.G_zm[0, 0] == pytest.approx(e["G_z_minus"], rel=1e-15)
    assert grid.G_zp[0, 0] == pytest.approx(e["G_z_plus"], rel=1e-15)
    assert grid.D0[0, 0] == pytest.approx(e["D0"], rel=1e-15)
    assert grid.mu[0, 0] == pytest.approx(e["mu"], rel=1e-15)
    assert grid.s_eps0[0, 0] == pytest.approx(e["s_times_eps0"], rel=1e-15)
    # the assembled row and right-hand side of the paper's Dirichlet cell equation
    A = fv.assemble(grid).toarray()
    assert A[0, 0] == pytest.approx(10.5, rel=1e-15)
    pb = np.zeros(grid.shape)
    pb[0, 1, 2] = 1.0  # prescribed east face value
    assert fv.rhs(grid, np.zeros(grid.shape), pb)[0] == pytest.approx(5.0, rel=1e-15)


def test_vertex_builder_reproduces_the_uniform_grid():
    u = fv.Grid(9, 4, 7, 0.02, 0.05, 0.05 / 6)
    v = fv.Grid.vertex(u.r, u.z, 4)
    for name in ("G_rm", "G_rp", "G_zm", "G_zp", "D0", "mu", "s_eps0"):
        np.testing.assert_allclose(getattr(v, name), getattr(u, name), rtol=1e-14, atol=0)


@pytest.mark.parametrize("beta", [1.0, 1.15])
def test_cell_centred_operator_is_spd_m_matrix(beta):
    g = fv.Grid.cell_centred(stretched(0.02, 0.05, 6, beta), stretched(0.0, 0.05, 5, 1 / beta), 5)
    A = fv.assemble(g).toarray()
    np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-15 * np.abs(A).max())
    assert np.linalg.eigvalsh(A).min() > 0
    off = A - np.diag(np.diag(A))
    assert (off <= 0).all()
    # weak diagonal dominance, strict in rows with a Dirichlet face
    assert (np.diag(A) + off.sum(axis=1) >= -1e-12 * np.abs(A).max()).all()


@pytest.mark.parametrize("builder", ["cell", "vertex"])
def test_dense_and_sparse_agree_on_stretched_grids(builder):
    rng = np.random.Generator(np.random.PCG64(3))
    if builder == "cell":
        g = fv.Grid.cell_centred(stretched(0.02, 0.05, 7, 1.2), stretched(0.0, 0.05, 6, 0.85), 6)
    else:
        g = fv.Grid.vertex(stretched(0.02, 0.05, 8, 1.2), stretched(0.0, 0.05, 7, 0.85), 6)
    rho = rng.standard_normal(g.shape) * 1e-6
    bc = (0.0, 1.0, -2.0, 300.0)
    a = solvers.solve_dense(g, rho, bc)
    b = solvers.solve_sparse(g, rho, bc)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-13


def test_mode_decomposition_is_exact_on_a_cell_centred_grid():
    """3-D dense solve vs the mode path (azimuthal DFT, per-plane direct solves of
    A_0 + lambda M, inverse DFT), written out here and as solvers.solve_modes."""
    rng = np.random.Generator(np.random.PCG64(5))
    g = fv.Grid.cell_centred(stretched(0.02, 0.05, 5, 1.3), stretched(0.0, 0.05, 4, 1.0), 6)
    rho = rng.standard_normal(g.shape) * 1e-6
    full = solvers.solve_dense(g, rho, (0.0, 0.0, 0.0, 0.0))
    b = fv.rhs(g, rho, np.zeros(g.shape)).reshape(g.interior_shape)
    planes = spectral.forward(b)
    lam = spectral.plane_eigenvalues(g.ntheta, float(g.dtheta))
    sol = np.zeros_like(planes)
    for p in range(g.ntheta):
        sol[p] = solvers.solve_mode(g, lam[p], planes[p].ravel()).reshape(planes[p].shape)
    back = spectral.inverse(sol)
    np.testing.assert_allclose(back, full[:, 1:-1, 1:-1], rtol=0, atol=1e-12 * np.abs(full).max())
    np.testing.assert_allclose(solvers.solve_modes(g, rho, (0.0, 0.0, 0.0, 0.0)), full, rtol=0,
                               atol=1e-12 * np.abs(full).max())


@pytest.mark.parametrize("builder,ntheta", [("cell", 7), ("vertex", 8)])
def test_solve_modes_matches_the_sparse_3d_solve_with_boundary_data(builder, ntheta):
    rng = np.random.Generator(np.random.PCG64(8))
    if builder == "cell":
        g = fv.Grid.cell_centred(stretched(0.02, 0.05, 9, 1.15), stretched(0.0, 0.05, 11, 0.9), ntheta)
    else:
        g = fv.Grid.vertex(stretched(0.02, 0.05, 12, 0.9), stretched(0.0, 0.05, 10, 1.2), ntheta)
    rho = rng.standard_normal(g.shape) * 1e-6
    bc = (5.0, -3.0, 1.0, 200.0)
    a = solvers.solve_sparse(g, rho, bc)
    b = solvers.solve_modes(g, rho, bc)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-13


def _manufactured_axisymmetric(r, z, r_in, W, L):
    """phi = sin(pi (r - r_in)/W) sin(pi z / L), zero on the boundary, and
    rho = -eps0 * Laplacian(phi) in cylindrical coordinates (m = 0)."""
    a, b = math.pi / W, math.pi / L
    f = np.sin(a * (r - r_in))
    fp = a * np.cos(a * (r - r_in))
    gz = np.sin(b * z)
    lap = (-a * a * f + fp / r - b * b * f)[None, :] * gz[:, None]
    return f[None, :] * gz[:, None], -EPS0 * lap


@pytest.mark.parametrize("beta", [1.0, 1.1])
def test_cell_centred_scheme_is_second_order(beta):
    r_in, r_out, L = 0.02, 0.05, 0.05
    errs = []
    for n in (8, 16, 32):
        # refine a stretched mesh by splitting every cell (keeps the stretching smooth)
        rf = stretched(r_in, r_out, n, beta ** (8 / n))
        zf = stretched(0.0, L, n, 1.0)
        g = fv.Grid.cell_centred(rf, zf, 1)
        phi, rho2 = _manufactured_axisymmetric(g.r, g.z, r_in, r_out - r_in, L)
        rho = np.zeros(g.shape)
        rho[0] = rho2
        u = solvers.solve_sparse(g, rho, (0.0, 0.0, 0.0, 0.0))
        e = u[0, 1:-1, 1:-1] - phi[1:-1, 1:-1]
        errs.append(np.sqrt((e ** 2).mean()) / np.sqrt((phi[1:-1, 1:-1] ** 2).mean()))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.7 < r2 < 4.3, errs


def test_max_principle_on_a_stretched_cell_centred_grid():
    g = fv.Grid.cell_centred(stretched(0.02, 0.05, 8, 1.25), stretched(0.0, 0.05, 8, 0.8), 4)
    u = solvers.solve_sparse(g, np.zeros(g.shape), (3.0, 7.0, 1.0, 300.0))
    assert u[:, 1:-1, 1:-1].min() >= 1.0 - 1e-9 and u[:, 1:-1, 1:-1].max() <= 300.0 + 1e-9
