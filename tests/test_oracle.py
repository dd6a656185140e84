"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage or fact it checks.  None compares the oracle with
itself by retyping a formula: the pins are printed worked examples, closed
forms checked numerically, library routines, brute force, exact special
solutions, and the second-order convergence of the discretisation to an
analytic solution of the differential equation.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import fv, solvers, spectral

INTERIOR = (slice(None), slice(1, -1), slice(1, -1))


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


# ---------------------------------------------------------------- App. A pins
def test_worked_cell_coefficients(golden_dir):
    """App. A worked five-point stencil: G = (1.5, 2.5, 2, 2), mu = 0.5, s = 2/eps0, D0 = 8."""
    g = json.load(open(os.path.join(golden_dir, "appendix_a_worked_cell.json")))
    c = fv.cell_coefficients(**g["input"])
    for key, val in g["expected"].items():
        assert c[key] == pytest.approx(val, rel=1e-15), key
    assert fv.charge_scale(c) == pytest.approx(2.0 / fv.EPS0, rel=1e-15)
    row = [c["D0"], -c["G_rm"], -c["G_rp"], -c["G_zm"], -c["G_zp"]]
    assert row == pytest.approx(g["matrix_row"]["entries_at_lambda_0"], rel=1e-15)
    assert c["mu"] == pytest.approx(g["matrix_row"]["centre_per_unit_lambda"])
    # the cell widths are the face differences (Eq. cell_geometry_appendix)
    assert g["input"]["r_hi"] - g["input"]["r_lo"] == g["input"]["dr"]


def test_two_cell_shifted_matrix(golden_dir):
    """App. A two-cell example: A_m = A_0 + lambda M gives [[9.5, -2], [-2, 10.2]] at lambda = 3."""
    g = json.load(open(os.path.join(golden_dir, "appendix_a_two_cell.json")))
    Am = solvers.mode_operator(np.array(g["A0"]), np.array(g["mu"]), g["lambda"]).toarray()
    np.testing.assert_allclose(Am, g["expected_Am"], rtol=1e-15)


# ------------------------------------------------------- eigenvalue and DFT
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 16, 128])
def test_eigenvalue_diagonalises_periodic_difference(n):
    """Eq. (discrete_azimuthal_eigenvalue): -delta_aa e^{i theta_m j} = lambda_m e^{i theta_m j}."""
    dth = 2 * math.pi / n
    j = np.arange(n)
    C = np.zeros((n, n))
    for a in range(n):
        C[a, a] += 2.0
        C[a, (a + 1) % n] -= 1.0
        C[a, (a - 1) % n] -= 1.0
    C /= dth * dth
    for m in range(n):
        v = np.exp(1j * 2 * math.pi * m * j / n)
        lam = spectral.discrete_eigenvalue(m, n, dth)
        np.testing.assert_allclose(C @ v, lam * v, atol=1e-12 * max(1.0, lam))
    ev = np.sort(np.linalg.eigvalsh(C))
    np.testing.assert_allclose(np.sort(spectral.discrete_eigenvalue(np.arange(n), n, dth)), ev,
                               atol=1e-11 * ev.max() if n > 1 else 1e-12)
    # not the continuous k_m^2 (the paper's point): differs at finite resolution
    if n >= 8:
        m = n // 2
        assert abs(spectral.discrete_eigenvalue(m, n, dth) - m * m) > 0.1 * m * m


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 16])
def test_planes_match_numpy_rfft(n):
    """Planes are Re and Im of numpy.fft.rfft / N (Eq. azimuthal_dft, R2C count of Sec. 3.1)."""
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, 3, 5))
    P = spectral.forward(x)
    F = np.fft.rfft(x, axis=0) / n
    nc = n // 2 + 1
    np.testing.assert_allclose(P[:nc], F.real, atol=1e-15)
    np.testing.assert_allclose(P[nc:], F.imag[1:n - nc + 1], atol=1e-15)
    np.testing.assert_allclose(spectral.inverse(P), x, atol=1e-14)
    np.testing.assert_allclose(spectral.inverse(P), np.fft.irfft(F * n, n=n, axis=0), atol=1e-14)
    w = spectral.parseval_weights(n)
    assert np.sum(x * x) == pytest.approx(n * np.sum(w[:, None, None] * P * P), rel=1e-13)
    # plane modes: every m of 0..floor(n/2) once as cos, 1..ceil(n/2)-1 once as sin
    assert sorted(spectral.plane_modes(n)[:nc]) == list(range(nc))
    assert spectral.plane_is_sine(n).sum() == n - nc


# ------------------------------------------------------------- assembly pins
@pytest.mark.parametrize("shape", [(5, 4, 6), (3, 1, 3), (4, 2, 3), (6, 3, 5)])
def test_assembly_symmetric_m_matrix(shape):
    """App. A: positive diagonal, non-positive couplings (the sign note after Eq. radial_flux_balance),
    symmetric, weakly diagonally dominant and strictly so next to a Dirichlet face."""
    nr, nt, nz = shape
    g = fv.Grid(nr, nt, nz, 0.02, 0.05, 0.01)
    A = fv.assemble(g).toarray()
    np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-15 * np.abs(A).max())
    off = A - np.diag(np.diag(A))
    assert (np.diag(A) > 0).all() and (off <= 0).all()
    rows = A.sum(axis=1)
    assert (rows >= -1e-14 * np.abs(A).max()).all()
    assert np.linalg.eigvalsh(A).min() > 0  # SPD


@pytest.mark.parametrize("shape", [(6, 5, 7), (3, 1, 4), (5, 2, 3)])
def test_operator_annihilates_constant_and_axial_linear(shape):
    """The cell balance has zero net flux for a constant potential, and for phi = a + b z
    the two axial fluxes cancel (equal conductances, equal spacing)."""
    nr, nt, nz = shape
    g = fv.Grid(nr, nt, nz, 0.02, 0.05, 0.01, dtype=np.longdouble)
    ones = np.ones(g.shape, dtype=np.longdouble)
    scale = float(np.abs(g.D0).max())
    assert float(np.abs(fv.apply_full(g, 7.0 * ones)).max()) < 1e-16 * scale * 7
    lin = 3.0 + 5.0 * g.z[None, :, None] * ones
    assert float(np.abs(fv.apply_full(g, lin)).max()) < 1e-16 * scale * 8


def test_constant_and_linear_dirichlet_data_reproduced():
    """Special solutions: all faces at V gives phi = V; boundary data 300 z/L (non-constant
    on the radial faces) gives phi = 300 z/L, pinning every Dirichlet term b^D."""
    p = W.SMALL.with_sizes(9, 5, 8)
    g = fv.Grid.of(p)
    zero = np.zeros(g.shape)
    u = solvers.solve_sparse(g, zero, bc=(4.0, 4.0, 4.0, 4.0))
    np.testing.assert_allclose(u, 4.0, rtol=0, atol=1e-13)
    lin = np.broadcast_to(300.0 * g.z[None, :, None] / (g.dz * (g.nz - 1)), g.shape).copy()
    u = solvers.solve_sparse(g, zero, phi_boundary=lin)
    np.testing.assert_allclose(u, lin, rtol=0, atol=1e-11)


def _analytic(r_in, r_out, length):
    """phi_c = 100 z/L + 20 ln(r/r_in) + 50 R(r) Z(z) T(theta) and rho_c = -eps0 lap(phi_c)."""
    W_ = r_out - r_in
    a, b = math.pi / W_, math.pi / length

    def phi(T, Z, R):
        Rr = np.sin(a * (R - r_in))
        Zz = np.sin(b * Z)
        Tt = 1 + 0.5 * np.cos(2 * T) + 0.3 * np.sin(3 * T)
        return 100 * Z / length + 20 * np.log(R / r_in) + 50 * Rr * Zz * Tt

    def rho(T, Z, R):
        Rr = np.sin(a * (R - r_in))
        dR = a * np.cos(a * (R - r_in))
        d2R = -a * a * Rr
        Zz = np.sin(b * Z)
        d2Z = -b * b * Zz
        Tt = 1 + 0.5 * np.cos(2 * T) + 0.3 * np.sin(3 * T)
        d2T = -2.0 * np.cos(2 * T) - 2.7 * np.sin(3 * T)
        lap = 50 * ((d2R + dR / R) * Zz * Tt + Rr * d2Z * Tt + Rr * Zz * d2T / (R * R))
        return -fv.EPS0 * lap

    return phi, rho


def _convergence_errors(sizes, r_in=0.02, r_out=0.05, length=0.05):
    phi_c, rho_c = _analytic(r_in, r_out, length)
    errs = []
    for nr, nt, nz in sizes:
        g = fv.Grid(nr, nt, nz, r_in, r_out, length / (nz - 1))
        T = (2 * math.pi * np.arange(nt) / nt)[:, None, None]
        Z = g.z[None, :, None]
        R = g.r[None, None, :]
        exact = phi_c(T, Z, R) * np.ones(g.shape)
        u = solvers.solve_sparse(g, rho_c(T, Z, R) * np.ones(g.shape), phi_boundary=exact)
        errs.append(np.abs(u - exact).max())
    return np.array(errs)


CONV_SIZES = [(9, 16, 9), (17, 32, 17), (33, 64, 33)]


@pytest.mark.slow
def test_second_order_convergence_to_analytic_solution():
    """The discrete solution converges at second order to a solution of Eq. (cylindrical_poisson)
    with radial, axial and azimuthal structure and non-constant Dirichlet data.  A dropped or
    mis-signed term, a wrong face radius or a missing eps0 leaves an O(1) error instead."""
    e = _convergence_errors(CONV_SIZES)
    ratios = e[:-1] / e[1:]
    assert e[-1] < 0.15  # volts, against |phi| up to ~170
    assert (ratios > 3.8).all() and (ratios < 4.2).all(), (e, ratios)


@pytest.mark.slow
@pytest.mark.parametrize("mutation", ["swap_radial_faces", "drop_theta", "flip_theta_sign", "node_radius_for_mu"])
def test_convergence_pin_catches_planted_mistakes(monkeypatch, mutation):
    """Plant a plausible mistake in the oracle (CPU only) and check the convergence pin fails."""
    orig = fv.cell_coefficients

    def mutated(r_lo, r_hi, r_c, dr, dz, d_w, d_e, d_s, d_n):
        c = orig(r_lo, r_hi, r_c, dr, dz, d_w, d_e, d_s, d_n)
        if mutation == "swap_radial_faces":
            c = orig(r_hi, r_lo, r_c, dr, dz, d_w, d_e, d_s, d_n)
        elif mutation == "drop_theta":
            c["mu"] = 0 * c["mu"]
        elif mutation == "flip_theta_sign":
            c["mu"] = -c["mu"]
        elif mutation == "node_radius_for_mu":
            c["mu"] = dr * dz * r_c / (0.02 * 0.02)
        return c

    monkeypatch.setattr(fv, "cell_coefficients", mutated)
    e = _convergence_errors(CONV_SIZES[:2])
    ratio = e[0] / e[1]
    assert not (3.8 < ratio < 4.2 and e[-1] < 0.5), (mutation, e)


# --------------------------------------------------------------- solver pins
TINY = [(3, 1, 3), (3, 4, 5), (5, 1, 3), (4, 2, 4), (5, 3, 4), (6, 5, 5), (7, 6, 6), (5, 8, 7)]


@pytest.mark.parametrize("shape", TINY)
def test_sparse_and_separable_match_dense(shape):
    """Brute force: dense LU of the assembled 3-D system vs SuperLU and the separable solver,
    including odd Ntheta, Ntheta in {1, 2} and single interior rows/columns."""
    nr, nt, nz = shape
    p = W.SMALL.with_sizes(nr, nt, nz)
    g = fv.Grid.of(p)
    rho = W.blob_charge(p, seed=nr * 100 + nt * 10 + nz)
    d = solvers.solve_dense(g, rho, p.bc)
    assert rel(solvers.solve_sparse(g, rho, p.bc), d) < 1e-14
    assert rel(solvers.solve_separable(g, rho, p.bc), d) < 1e-14
    # the dense solution satisfies every cell balance
    assert solvers.residual_norm(fv.Grid.of(p, np.longdouble), d, rho, p.bc) < 1e-14


@pytest.mark.parametrize("prob", [W.SMALL, W.HIGH_SHIFT.with_sizes(17, 64, 19)])
def test_separable_matches_sparse_direct(prob):
    """The separable exact solver agrees with the undecomposed sparse direct solve."""
    g = fv.Grid.of(prob)
    rho = W.blob_charge(prob, seed=3)
    assert rel(solvers.solve_separable(g, rho, prob.bc)[INTERIOR],
               solvers.solve_sparse(g, rho, prob.bc)[INTERIOR]) < 1e-13


@pytest.mark.slow
def test_separable_matches_sparse_direct_on_the_127k_proxy():
    """The separable solver, the reference for the large grids, against SuperLU
    on the undecomposed 3-D system at 63 x 32 x 63 interior nodes (127,008
    unknowns, the largest size sparse LU finishes in about a minute)."""
    p = W.BATCHED.with_sizes(65, 32, 65)
    g = fv.Grid.of(p)
    rho = W.blob_charge(p, seed=24680)
    sep = solvers.solve_separable(g, rho, p.bc)
    ref = solvers.solve_sparse(g, rho, p.bc)
    assert rel(sep[INTERIOR], ref[INTERIOR]) < 1e-13
    assert np.abs(sep - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("prob", [W.SMALL.with_sizes(17, 8, 19), W.HIGH_SHIFT.with_sizes(17, 7, 13)])
def test_extended_precision_separable_is_exact(prob):
    """Run in extended precision, the separable solver leaves a relative residual
    of the assembled cell balances (evaluated by apply_full in extended
    precision, code the solver does not use) at the extended-precision level,
    and agrees with the FP64 sparse direct solve to FP64 rounding."""
    gl = fv.Grid.of(prob, np.longdouble)
    rho = W.blob_charge(prob, seed=8)
    ex = solvers.solve_separable(gl, rho, prob.bc)
    assert ex.dtype == np.longdouble
    eps_ld = float(np.finfo(np.longdouble).eps)
    assert solvers.residual_norm(gl, ex, rho, prob.bc) < 1e3 * eps_ld
    ref = solvers.solve_sparse(fv.Grid.of(prob), rho, prob.bc)
    assert rel(ex.astype(np.float64)[INTERIOR], ref[INTERIOR]) < 1e-14
    # the FP64 run of the same solver is not that exact: its residual is at FP64 level
    f64 = solvers.solve_separable(fv.Grid.of(prob), rho, prob.bc)
    assert solvers.residual_norm(gl, f64, rho, prob.bc) > 1e2 * eps_ld


@pytest.mark.parametrize("n", [1, 2, 5, 16, 128])
def test_extended_precision_eigenvalue_matches_fp64(n):
    """Eq. discrete_azimuthal_eigenvalue in extended precision agrees with FP64 to rounding."""
    dth = 2.0 * math.pi / n
    m = np.arange(n)
    ld = spectral.discrete_eigenvalue(m, n, np.longdouble(2) * np.arccos(np.longdouble(-1)) / n,
                                      dtype=np.longdouble)
    assert ld.dtype == np.longdouble
    np.testing.assert_allclose(ld.astype(np.float64), spectral.discrete_eigenvalue(m, n, dth),
                               rtol=1e-14, atol=1e-14 * float(ld.max() if n > 1 else 1.0))


@pytest.mark.parametrize("shape", [(7, 6, 6), (6, 5, 7), (5, 2, 5), (5, 1, 4)])
def test_mode_decomposition_is_exact(shape):
    """Sec. 3.1-3.2: DFT in theta, the 2-D systems (A_0 + lambda_m M) u = s rho^ + b^D delta_{m0}
    per plane, inverse DFT == the undecomposed 3-D dense solve (to rounding)."""
    nr, nt, nz = shape
    p = W.HIGH_SHIFT.with_sizes(nr, nt, nz)
    g = fv.Grid.of(p)
    rho = W.blob_charge(p, seed=11)
    full = solvers.solve_dense(g, rho, p.bc)
    b = fv.rhs(g, rho, fv.boundary_values(g, p.bc))
    bh = spectral.forward(b)
    lam = spectral.plane_eigenvalues(nt, float(g.dtheta))
    uh = np.stack([solvers.solve_mode(g, lam[q], bh[q]) for q in range(nt)])
    u = spectral.inverse(uh)
    assert rel(u, full[INTERIOR]) < 1e-14
    # the boundary term enters only the m = 0 plane (Eq. mode_rhs)
    bd = fv.rhs(g, np.zeros(g.shape), fv.boundary_values(g, p.bc))
    pd = spectral.forward(bd)
    if nt > 1:
        assert np.abs(pd[1:]).max() < 1e-12 * np.abs(pd[0]).max()


def test_manufactured_recovery_small():
    """phi_true is recovered from rho = A phi_true / s (formed in extended precision) to ~1e-15."""
    p = W.SMALL
    phit = W.manufactured_potential(p, 12345, np.longdouble)
    rho = fv.charge_from_potential(fv.Grid.of(p, np.longdouble), phit).astype(np.float64)
    u = solvers.solve_sparse(fv.Grid.of(p), rho, p.bc)
    assert rel(u[INTERIOR], phit.astype(np.float64)[INTERIOR]) < 1e-14
    np.testing.assert_array_equal(u[:, 0, :], p.phi_z0)
    np.testing.assert_array_equal(u[:, -1, :], p.phi_zL)
    np.testing.assert_array_equal(u[:, 1:-1, 0], p.phi_r_in)


def test_discrete_maximum_principle():
    """M-matrix: with rho = 0 the solution lies between the smallest and largest boundary values."""
    p = W.SMALL.with_sizes(17, 8, 17)
    u = solvers.solve_sparse(fv.Grid.of(p), np.zeros(p.shape), p.bc)
    inner = u[INTERIOR]
    assert inner.min() > 0.0 and inner.max() < 300.0
    # theta-invariant data gives a theta-invariant solution
    assert np.abs(inner - inner[:1]).max() < 1e-12


def test_linearity_and_theta_reflection():
    p = W.SMALL.with_sizes(9, 7, 10)
    g = fv.Grid.of(p)
    r1, r2 = W.blob_charge(p, 1), W.blob_charge(p, 2)
    zero_bc = (0.0, 0.0, 0.0, 0.0)
    s1 = solvers.solve_sparse(g, r1, zero_bc)
    s2 = solvers.solve_sparse(g, r2, zero_bc)
    s12 = solvers.solve_sparse(g, 2.0 * r1 - 3.0 * r2, zero_bc)
    assert rel(s12, 2.0 * s1 - 3.0 * s2) < 1e-13
    # theta -> -theta: cos planes unchanged, sin planes negated, so the solution reflects
    refl = r1[(-np.arange(p.ntheta)) % p.ntheta]
    sr = solvers.solve_sparse(g, refl, zero_bc)
    assert rel(sr, s1[(-np.arange(p.ntheta)) % p.ntheta]) < 1e-13


def test_axisymmetric_reduces_to_one_plane():
    """Theta-invariant rho: the 3-D solution equals the Ntheta = 1 (m = 0 only) solve on every plane."""
    p = W.SMALL.with_sizes(11, 6, 9)
    rho1 = W.blob_charge(p.with_sizes(11, 1, 9), 5)
    rho = np.repeat(rho1, 6, axis=0)
    u = solvers.solve_sparse(fv.Grid.of(p), rho, p.bc)
    u1 = solvers.solve_sparse(fv.Grid.of(p.with_sizes(11, 1, 9)), rho1, p.bc)
    assert rel(u, np.repeat(u1, 6, axis=0)) < 1e-14


def test_extended_precision_apply_matches_assembled_matrix():
    """The stencil form (apply_full) and the assembled matrix agree: A_full phi = A u - b^D."""
    p = W.HIGH_SHIFT.with_sizes(7, 5, 6)
    g = fv.Grid.of(p)
    phi = W.manufactured_potential(p, 7)
    lhs = fv.apply_full(g, phi)
    A = fv.assemble(g)
    bd = fv.rhs(g, np.zeros(g.shape), phi)
    np.testing.assert_allclose(lhs.ravel(), A @ phi[INTERIOR].ravel() - bd.ravel(),
                               atol=1e-12 * np.abs(lhs).max())
    gl = fv.Grid.of(p, np.longdouble)
    ll = fv.apply_full(gl, phi.astype(np.longdouble))
    np.testing.assert_allclose(lhs, ll.astype(np.float64), atol=1e-13 * float(np.abs(ll).max()))
