"""Explicit meshes (App. A): cell-centred finite volumes with half-cell
Dirichlet faces, and vertex- or cell-centred grids with non-uniform r and z
spacing, solved through the C ABI and compared with the oracle's direct mode
solves (exact up to rounding) on the same seeded inputs."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fv, solvers

from gpu_util import INTERIOR, dev, host, rel_l2, say

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
BC = (5.0, -3.0, 1.0, 300.0)
ST = W.stretched_points

# name -> (layout, r, z, ntheta); r/z are node coordinates (vertex) or cell faces (cell)
CASES = {
    # uniform cells, register FFT, several fused chunks per plane and a ragged last chunk
    "cell_uniform": ("cell", np.linspace(0.02, 0.05, 97), np.linspace(0.0, 0.06, 131), 16),
    # cells stretched towards the inner wall and the top face, dense DFT path
    "cell_stretched": ("cell", ST(0.02, 0.05, 80, 1.015), ST(0.0, 0.06, 100, 0.985), 12),
    # non-uniform vertex-centred nodes
    "vertex_stretched": ("vertex", ST(0.02, 0.05, 71, 1.02), ST(0.0, 0.05, 90, 1.012), 16),
    # few cells: the coarsest (direct) level is the whole plane
    "cell_tiny": ("cell", ST(0.02, 0.05, 9, 1.1), ST(0.0, 0.02, 6, 1.0), 5),
    # odd counts, one level coarsened in r only (cells about 3:1)
    "cell_flat": ("cell", np.linspace(0.02, 0.05, 41), np.linspace(0.0, 0.12, 34), 6),
}


@pytest.fixture(scope="module")
def P():
    import paper_2609_07172_amd as P
    P.library()
    assert torch.cuda.is_available()
    return P


def layout_of(P, name):
    return P.CELL if name == "cell" else P.VERTEX


def oracle_grid(case):
    layout, r, z, nt = case
    return fv.Grid.cell_centred(r, z, nt) if layout == "cell" else fv.Grid.vertex(r, z, nt)


def plan_for(P, case, **options):
    layout, r, z, nt = case
    return P.Plan.from_mesh(r, z, nt, layout_of(P, layout), BC, **options)


_REF = {}


def reference(name):
    """Seeded charge on the mesh nodes and the oracle's solution (cached per case)."""
    if name not in _REF:
        g = oracle_grid(CASES[name])
        rho = W.mesh_blob_charge(g.r, g.z, g.ntheta, seed=len(name))
        _REF[name] = (g, rho, solvers.solve_modes(g, rho, BC))
    return _REF[name]


@pytest.mark.parametrize("name", list(CASES))
def test_mesh_solve_matches_oracle(P, name):
    g, rho, ref = reference(name)
    say("mesh solve", name, g.shape)
    plan = plan_for(P, CASES[name])
    assert plan.shape == g.shape
    info = plan.info()
    assert info["layout"] == layout_of(P, CASES[name][0]) and info["uniform"] == 0
    phi, st = plan.solve(dev(rho), tol=1e-13)
    say("cycles", st["cycles"])
    assert st["status"] == P.OK, st
    # point smoothing is weaker where the cells are stretched (about 30 cycles
    # at 6:1 spacing ratios, 8 to 12 on uniform cells)
    assert st["cycles"] <= 36, st["cycles"]
    got = host(phi)
    assert rel_l2(got, ref) <= 1e-12, rel_l2(got, ref)
    # boundary nodes carry the Dirichlet values (axial faces win at the corners)
    np.testing.assert_allclose(got[:, 1:-1, 0], BC[0], rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(got[:, 1:-1, -1], BC[1], rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(got[:, 0, :], BC[2], rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(got[:, -1, :], BC[3], rtol=1e-13, atol=1e-12)


def test_large_meshes_run_fused_passes(P):
    """Irregular rows next to the faces or everywhere (stretched z) no longer keep
    a level off the fused passes."""
    for name in ("cell_uniform", "cell_stretched", "vertex_stretched"):
        info = plan_for(P, CASES[name]).info()
        assert info["fused_levels"] >= 1, (name, info)


@pytest.mark.parametrize("options", [dict(fused=0), dict(precision=32), dict(masks=1), dict(groups=3),
                                     dict(graph=1), dict(nu1=1, nu2=3), dict(bottom=0)],
                         ids=lambda o: ",".join(f"{k}={v}" for k, v in o.items()))
def test_stretched_cells_every_solver_path(P, options):
    g, rho, ref = reference("cell_stretched")
    say("mesh options", options)
    plan = plan_for(P, CASES["cell_stretched"], **options)
    phi, st = plan.solve(dev(rho), tol=1e-13)
    assert st["status"] == P.OK, st
    assert rel_l2(host(phi), ref) <= 1e-12, rel_l2(host(phi), ref)


@pytest.mark.parametrize("name", ["cell_stretched", "vertex_stretched", "cell_uniform"])
@pytest.mark.parametrize("chunk,fmg", [(0, 0), (7, 0), (0, 1)])
def test_fused_passes_on_meshes_equal_the_per_step_kernels(P, name, chunk, fmg):
    """On a stretched mesh almost no two rows share their axial coefficients, so the
    fused passes take unchecked steps that form every row's coefficients from its
    tables; the iterates stay bitwise those of the one-kernel-per-step path (the
    merged finest pass included: no check falls between the first cycles).  The
    full-multigrid start needs the fused passes, so with it the reference is the
    fused path with two rows of prefetch: checked steps only, and a start that is
    written out instead of formed by the first down passes as they stream."""
    g, rho, _ = reference(name)
    say("fused-vs-step mesh", name, "chunk", chunk, "fmg", fmg)
    a = plan_for(P, CASES[name], fused=1, max_cycles=5, chunk_rows=chunk, chunk_rows_coarse=chunk,
                 chunk_rows_merge=chunk, fmg=fmg)
    b = plan_for(P, CASES[name], fused=0, max_cycles=5) if not fmg else \
        plan_for(P, CASES[name], fused=1, max_cycles=5, prefetch=2, fmg=1)
    pa, sa = a.solve(dev(rho), tol=1e-30, allow=(P.OK, P.NOT_CONVERGED))
    pb, sb = b.solve(dev(rho), tol=1e-30, allow=(P.OK, P.NOT_CONVERGED))
    assert sa["cycles"] == sb["cycles"] == 5
    np.testing.assert_array_equal(host(pa), host(pb))


def test_autotuner_picks_omega_on_a_stretched_mesh(P):
    """With option tune_omega the autotuner sets the over-relaxation factor from the
    measured contraction per cycle; on stretched cells the tuned plan needs no more
    cycles than the default for the same answer, and omega is one of its candidates."""
    g, rho, ref = reference("cell_stretched")
    say("tune omega", g.shape)
    _, st0 = plan_for(P, CASES["cell_stretched"]).solve(dev(rho), tol=1e-13)
    plan = plan_for(P, CASES["cell_stretched"], tune_omega=1)
    plan.autotune()
    w = plan.get_option("omega")
    say("omega", w, "default cycles", st0["cycles"])
    assert w in (1.0, 1.1, 1.15, 1.2, 1.25, 1.3, 1.35, 1.4, 1.5)
    phi, st = plan.solve(dev(rho), tol=1e-13)
    assert st["status"] == P.OK, st
    assert st["cycles"] <= st0["cycles"], (w, st["cycles"], st0["cycles"])
    assert rel_l2(host(phi), ref) <= 1e-12


def test_warm_start_on_a_mesh(P):
    g, rho, ref = reference("vertex_stretched")
    say("mesh warm start")
    plan = plan_for(P, CASES["vertex_stretched"])
    cold, st0 = plan.solve(dev(rho), tol=1e-13)
    plan.set_option("warm_start", 1)
    phi = cold.clone()
    phi, st1 = plan.solve(dev(rho * 1.001), tol=1e-13, phi=phi)
    assert st1["status"] == P.OK and st1["cycles"] < st0["cycles"], (st0["cycles"], st1["cycles"])
    ref2 = solvers.solve_modes(g, rho * 1.001, BC)
    assert rel_l2(host(phi), ref2) <= 1e-12


def test_uniform_mesh_matches_the_uniform_constructor(P):
    """The explicit-coordinate path on uniform vertex nodes gives the uniform plan's
    answer (tables differ only by the rounding of the coordinates)."""
    p = W.SMALL.with_sizes(65, 16, 49)
    say("uniform via mesh", p.shape)
    th, z, r = W.node_coordinates(p)
    rho = dev(W.blob_charge(p, seed=4))
    a, sa = P.Plan.for_problem(p).solve(rho, tol=1e-13)
    b, sb = P.Plan.from_mesh(r, z, p.ntheta, P.VERTEX, p.bc).solve(rho, tol=1e-13)
    assert sa["status"] == sb["status"] == P.OK
    assert abs(sa["cycles"] - sb["cycles"]) <= 1
    assert rel_l2(host(b), host(a)) <= 1e-12


def test_cell_centred_apply_matches_oracle(P):
    g, _, _ = reference("cell_stretched")
    say("mesh apply", g.shape)
    layout, r, z, nt = CASES["cell_stretched"]
    phi = np.zeros(g.shape)
    rng = np.random.Generator(np.random.PCG64(21))
    phi[INTERIOR] = rng.standard_normal(phi[INTERIOR].shape)
    phi[:, :, 0], phi[:, :, -1], phi[:, 0, :], phi[:, -1, :] = BC
    plan = plan_for(P, CASES["cell_stretched"])
    out = torch.empty_like(dev(phi))
    P.apply(plan.handle, dev(phi), out)
    got = host(out)
    gl = fv.Grid.cell_centred(np.asarray(r, np.longdouble), np.asarray(z, np.longdouble), nt, np.longdouble)
    ref = fv.charge_from_potential(gl, phi.astype(np.longdouble)).astype(np.float64)
    # bound: the size of the terms that cancel, |A| |phi| + |b^D| (|phi|), over s
    a = abs(fv.assemble(g))
    ab = np.abs(phi)
    scale = (a @ ab[INTERIOR].ravel() + fv.rhs(g, np.zeros(g.shape), ab).ravel()).reshape(g.interior_shape)
    scale = scale * fv.EPS0 / g.s_eps0
    col = scale.max(axis=0)[None] * nt
    err = np.abs(got[INTERIOR] - ref[INTERIOR])
    assert (err <= 64 * EPS * col).all(), float((err / col).max() / EPS)
    assert (got[:, 0, :] == 0).all() and (got[:, :, 0] == 0).all()


@pytest.mark.parametrize("name", ["cell_stretched", "vertex_stretched"])
def test_multigrid_preconditioned_fgmres_on_stretched_meshes(P, name):
    """One V-cycle as the FGMRES preconditioner: fewer V-cycles in all than the
    plain iteration where the point smoother is weak, same answer."""
    g, rho, ref = reference(name)
    say("mg-fgmres", name)
    _, s0 = plan_for(P, CASES[name]).solve(dev(rho), tol=1e-13)
    plan = plan_for(P, CASES[name], krylov=1, krylov_precond=3)
    phi, st = plan.solve(dev(rho), tol=1e-13)
    say("plain cycles", s0["cycles"], "fgmres steps", st["krylov_iterations"])
    assert st["status"] == P.OK and st["learned_fallback"] == 0, st
    assert st["cycles"] == st["krylov_iterations"]  # one preconditioning V-cycle per step
    assert rel_l2(host(phi), ref) <= 1e-12
    assert st["krylov_iterations"] < 0.75 * s0["cycles"], (st["krylov_iterations"], s0["cycles"])
    # the per-step contraction beats the plain iteration's mean contraction
    plain_rate = (s0["rel_residual"] / 1.0) ** (1.0 / s0["cycles"])
    assert st["learned_rate"] < plain_rate, (st["learned_rate"], plain_rate)


def test_masks_do_not_leak_into_a_later_fgmres_solve(P):
    """Planes frozen by a masked solve are not skipped by the V-cycles of a later
    FGMRES solve on the same plan."""
    g, rho, _ = reference("cell_uniform")
    # an axisymmetric charge: every plane but plane 0 starts within its share of
    # the tolerance and freezes at the first check
    rho = np.ascontiguousarray(np.broadcast_to(rho.mean(axis=0, keepdims=True), rho.shape))
    ref = solvers.solve_modes(g, rho, BC)
    say("masks then fgmres")
    plan = plan_for(P, CASES["cell_uniform"], masks=1)
    _, st = plan.solve(dev(rho), tol=1e-13)
    assert st["status"] == P.OK and st["frozen_planes"] > 0, st
    plan.set_option("krylov", 1)
    plan.set_option("krylov_precond", 3)
    phi, st = plan.solve(dev(rho), tol=1e-13)
    assert st["status"] == P.OK, st
    assert rel_l2(host(phi), ref) <= 1e-12


def test_paper_scale_stretched_cells_sampled_planes(P):
    """400 x 128 x 512 nodes on cells stretched 4:1 towards the inner wall and
    z = 0: three Fourier planes of the GPU solution (the GPU's own forward DFT
    of phi) against the oracle's direct solves of those modes.  Per-plane
    errors are bounded by the field's (Parseval), so each must be within
    1e-12 of the interior field norm.  All 128 planes: the residual of every
    mode equation for the oracle's DFT of the answer."""
    nr, nt, nz = 400, 128, 512
    rf = W.stretched_points(0.02, 0.05, nr - 2, 4.0 ** (1.0 / (nr - 3)))
    zf = W.stretched_points(0.0, 0.1, nz - 2, 0.25 ** (1.0 / (nz - 3)))
    g = fv.Grid.cell_centred(rf, zf, nt)
    rho = W.mesh_blob_charge(g.r, g.z, nt, seed=3)
    bc = (0.0, 0.0, 0.0, 300.0)
    say("paper-scale stretched cells", g.shape)
    plan = P.Plan.from_mesh(rf, zf, nt, P.CELL, bc)
    phi_d, st = plan.solve(dev(rho), tol=1e-13)
    assert st["status"] == P.OK, st
    planes_d = torch.empty_like(phi_d)
    P.dft_forward(plan.handle, phi_d, planes_d)
    got = host(planes_d)
    phi = host(phi_d)
    from oracle import spectral
    b = fv.rhs(g, rho, fv.boundary_values(g, bc))
    bp = spectral.forward(np.reshape(b, g.interior_shape))
    lam = spectral.plane_eigenvalues(nt, float(g.dtheta))
    norm = np.linalg.norm(phi[INTERIOR])
    for p in (0, 1, 100):  # m = 0 (with the boundary term), cos m = 1, sin m = 37
        ref = solvers.solve_mode(g, lam[p], bp[p].ravel())
        err = np.linalg.norm(got[p, 1:-1, 1:-1] - ref) * np.sqrt(nt)
        say("plane", p, err / norm)
        assert err <= 1e-12 * norm, (p, err / norm)
    # every plane at full size: the oracle's own DFT of the answer satisfies each
    # mode equation (A_0 + lambda_p M) u_p = b_p to the solve's tolerance (the
    # library weighs the planes as Parseval does, within a factor of 2 of this sum)
    up = spectral.forward(phi[:, 1:-1, 1:-1])
    A0 = solvers.plane_matrix(g)
    r2 = b2 = 0.0
    for p in range(nt):
        r = bp[p].ravel() - solvers.mode_operator(A0, g.mu, float(lam[p])) @ up[p].ravel()
        r2 += float(r @ r)
        b2 += float(bp[p].ravel() @ bp[p].ravel())
    rel = np.sqrt(r2 / b2)
    say("all-plane relative residual", rel, "library", st["rel_residual"])
    assert rel <= 3e-13, rel


@pytest.mark.parametrize("smoother", [1, 2])
@pytest.mark.parametrize("name", ["cell_stretched", "vertex_stretched", "cell_flat", "cell_tiny"])
def test_line_smoothers_match_oracle(P, name, smoother):
    """Zebra line relaxation (r-lines; alternating r- and z-lines) reaches the
    oracle's answer; it runs on the one-kernel-per-colour path."""
    g, rho, ref = reference(name)
    say("line smoother", smoother, name)
    plan = plan_for(P, CASES[name], smoother=smoother)
    assert plan.info()["fused_levels"] == 0 and plan.get_option("smoother") == smoother
    phi, st = plan.solve(dev(rho), tol=1e-13)
    say("cycles", st["cycles"])
    assert st["status"] == P.OK, st
    assert rel_l2(host(phi), ref) <= 1e-12, rel_l2(host(phi), ref)


@pytest.mark.parametrize("name", ["cell_stretched", "vertex_stretched"])
def test_alternating_lines_need_fewer_cycles_on_stretched_meshes(P, name):
    g, rho, ref = reference(name)
    _, point = plan_for(P, CASES[name]).solve(dev(rho), tol=1e-13)
    _, lines = plan_for(P, CASES[name], smoother=2).solve(dev(rho), tol=1e-13)
    say(name, "point", point["cycles"], "alternating lines", lines["cycles"])
    assert lines["cycles"] < point["cycles"], (lines["cycles"], point["cycles"])


def test_line_smoother_on_the_uniform_grid_and_in_fgmres(P):
    p = W.SMALL
    rho = W.blob_charge(p, seed=8)
    ref = solvers.solve_sparse(fv.Grid.of(p), rho, p.bc)
    say("line smoother uniform")
    for opts in (dict(smoother=1), dict(smoother=2, krylov=1, krylov_precond=3)):
        phi, st = P.Plan.for_problem(p, **opts).solve(dev(rho), tol=1e-13)
        assert st["status"] == P.OK, (opts, st)
        assert rel_l2(host(phi), ref) <= 1e-12, (opts, rel_l2(host(phi), ref))


def test_smoother_option_errors(P):
    plan = P.Plan.for_problem(W.SMALL)
    for bad in (-1, 3, 1.5):
        with pytest.raises(P.CylPoissonError) as e:
            plan.set_option("smoother", bad)
        assert e.value.status == P.EINVAL
    plan.set_option("smoother", 1)
    plan.set_option("precision", 32)
    with pytest.raises(P.CylPoissonError) as e:
        plan.solve(dev(np.zeros(W.SMALL.shape)), tol=1e-12)
    assert e.value.status == P.EINVAL


# near-isotropic cells (dr ~ dz = 3e-5 m) so that FP64 resolves the answer to
# far below 1e-12; extremely flat cells put the oracle's own residual near 1e-11
LONG_LINES = {"long-r-lines": W.Problem(1030, 2, 9, 0.02, 0.05, 3e-5, name="long-r"),
              "long-z-lines": W.Problem(9, 2, 1030, 0.02, 0.02 + 8 * 3e-5, 3e-5, name="long-z")}


@pytest.mark.parametrize("name", list(LONG_LINES))
def test_long_lines_use_the_thomas_sweeps(P, name):
    """Lines longer than 1024 unknowns (past one workgroup of cyclic reduction)
    are solved by a Thomas sweep per thread; the result is the oracle's."""
    p = LONG_LINES[name]
    rho = W.blob_charge(p, seed=5)
    ref = solvers.solve_separable(fv.Grid.of(p), rho, p.bc)
    say("long lines", name, p.shape)
    for sm in (1, 2):
        phi, st = P.Plan.for_problem(p, smoother=sm).solve(dev(rho), tol=1e-13)
        assert st["status"] == P.OK, (sm, st)
        assert rel_l2(host(phi), ref) <= 1e-12, (sm, rel_l2(host(phi), ref))


# flat cells (34:1 and 1:34): FP64 cannot represent the answer to a 1e-13
# residual here (the exact solution rounded to FP64 leaves 1.8e-13 on the
# r-line grid), so the tolerance is derived from that floor
FLAT_LINES = {"long-r-lines-flat": W.Problem(1030, 2, 9, 0.02, 0.05, 1e-3, name="long-r-flat"),
              "long-z-lines-flat": W.Problem(9, 2, 1030, 0.02, 0.02 + 8e-3, 3e-5, name="long-z-flat")}


@pytest.mark.parametrize("name", list(FLAT_LINES))
def test_long_lines_on_flat_cells_reach_the_fp64_floor(P, name):
    """The Thomas-sweep line smoothers on lines longer than 1024 with flat cells.
    The tolerance is 3 times the relative residual of the exact discrete
    solution (the oracle's separable solve in extended precision) rounded to
    FP64, the smallest residual any FP64 answer can have; the answer must then
    lie within 1e-12 of the exact one, or within 30 times the oracle's own FP64
    error if that is larger."""
    p = FLAT_LINES[name]
    rho = W.blob_charge(p, seed=5)
    gl = fv.Grid.of(p, np.longdouble)
    exact = solvers.solve_separable(gl, rho, p.bc)
    floor = solvers.residual_norm(gl, exact.astype(np.float64), rho, p.bc)
    exact = exact.astype(np.float64)
    err64 = rel_l2(solvers.solve_separable(fv.Grid.of(p), rho, p.bc), exact)
    tol = 3.0 * max(floor, 1e-16)
    bound = max(1e-12, 30.0 * err64)
    say("flat long lines", name, p.shape, "tol", tol, "bound", bound)
    for sm in (1, 2):
        phi, st = P.Plan.for_problem(p, smoother=sm).solve(dev(rho), tol=tol)
        assert st["status"] == P.OK, (sm, st)
        assert rel_l2(host(phi), exact) <= bound, (sm, rel_l2(host(phi), exact))


def test_plans_reject_geometry_beyond_the_double_range(P):
    """Finite inputs whose finite-volume coefficients overflow are refused."""
    with pytest.raises(P.CylPoissonError) as e:
        P.Plan(5, 2, 5, 1.0, 1e300, 1e300)
    assert e.value.status == P.EINVAL and "non-finite" in P.last_error()
    with pytest.raises(P.CylPoissonError):
        P.Plan.from_mesh([1.0, 1e300, 1.5e300], [0.0, 1e300, 1.5e300], 2, P.VERTEX)
