"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances:
* DFT: each plane value is a sum of N terms of size |x_j|/N; two FP64
  evaluations differ by at most a few eps * sum_j |x_j| (per column).
* apply: the operator cancels large neighbour terms, so the bound is taken
  relative to the absolute-valued operator |A| |phi| / s at the node
  (times the column mixing of the two transforms).
* solve: relative L2 over interior nodes <= 1e-12 against the oracle's direct
  solution (the stated target); boundary nodes must equal the Dirichlet data.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fv, solvers, spectral

from gpu_util import INTERIOR, dev, histories_agree, host, rel_l2, say

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def P():
    import paper_2609_07172_amd as P
    P.library()
    assert torch.cuda.is_available()
    return P


def manufactured(p, seed=12345):
    """phi_true and rho = A phi_true / s formed in extended precision, rounded once."""
    phit = W.manufactured_potential(p, seed, np.longdouble)
    rho = fv.charge_from_potential(fv.Grid.of(p, np.longdouble), phit).astype(np.float64)
    return phit.astype(np.float64), rho


def check_boundary(phi, p):
    np.testing.assert_array_equal(phi[:, 0, :], p.phi_z0)
    np.testing.assert_array_equal(phi[:, -1, :], p.phi_zL)
    np.testing.assert_array_equal(phi[:, 1:-1, 0], p.phi_r_in)
    np.testing.assert_array_equal(phi[:, 1:-1, -1], p.phi_r_out)


# ------------------------------------------------------------------ DFT
@pytest.mark.parametrize("shape", [(5, 16, 7), (9, 7, 4), (6, 1, 5), (4, 2, 6), (33, 128, 9), (7, 32, 5),
                                   (11, 64, 13), (40, 128, 33)])
def test_dft_matches_oracle(P, shape):
    nr, nt, nz = shape
    say("dft", shape)
    plan = P.Plan(nr, nt, nz, 0.02, 0.05, 0.01)
    x = np.random.default_rng(nr + nt).standard_normal((nt, nz, nr))
    xd = dev(x)
    planes = torch.empty_like(xd)
    P.dft_forward(plan.handle, xd, planes)
    ref = spectral.forward(x)
    bound = 4 * EPS * np.abs(x).sum(axis=0)[None] + 1e-300
    err = np.abs(host(planes) - ref)
    assert (err <= bound).all(), float((err / bound).max())
    back = torch.empty_like(xd)
    P.dft_inverse(plan.handle, planes, back)
    ref_back = spectral.inverse(host(planes))
    bound = 8 * nt * EPS * np.abs(host(planes)).sum(axis=0)[None] + 1e-300
    assert (np.abs(host(back) - ref_back) <= bound).all()
    np.testing.assert_allclose(host(back), x, atol=64 * nt * EPS * np.abs(x).max())


# ---------------------------------------------------------------- apply
def abs_operator_scale(p, phi):
    """(|A| |phi| + |b^D|(|phi|)) / s at interior nodes: the size of the terms that cancel."""
    g = fv.Grid.of(p)
    a = abs(fv.assemble(g))
    ab = np.abs(phi)
    s = a @ ab[INTERIOR].ravel() + fv.rhs(g, np.zeros(g.shape), ab).ravel()
    return s.reshape(g.interior_shape) * fv.EPS0 / g.s_eps0


@pytest.mark.parametrize("prob", [W.SMALL, W.HIGH_SHIFT.with_sizes(17, 12, 13), W.SMALL.with_sizes(6, 5, 4)])
def test_apply_matches_oracle(P, prob):
    say("apply", prob.name, prob.shape)
    phi = W.manufactured_potential(prob, 3)
    plan = P.Plan.for_problem(prob)
    out = torch.empty_like(dev(phi))
    P.apply(plan.handle, dev(phi), out)
    got = host(out)
    ref = fv.charge_from_potential(fv.Grid.of(prob, np.longdouble), phi.astype(np.longdouble))
    ref = ref.astype(np.float64)
    scale = abs_operator_scale(prob, phi)
    col = scale.max(axis=0)[None] * prob.ntheta
    err = np.abs(got[INTERIOR] - ref[INTERIOR])
    assert (err <= 64 * EPS * col).all(), float((err / col).max() / EPS)
    assert (got[:, 0, :] == 0).all() and (got[:, -1, :] == 0).all()
    assert (got[:, :, 0] == 0).all() and (got[:, :, -1] == 0).all()


# ---------------------------------------------------------------- solve
def test_solve_small_matches_sparse_direct(P):
    """Small workload: 33 x 16 x 33, manufactured rho, against SuperLU of the 3-D system."""
    p = W.SMALL
    phit, rho = manufactured(p)
    ref = solvers.solve_sparse(fv.Grid.of(p), rho, p.bc)
    say("solve", p.name)
    plan = P.Plan.for_problem(p)
    phi, st = plan.solve(dev(rho), tol=1e-14)
    got = host(phi)
    assert st["status"] == P.OK and st["rel_residual"] <= 1e-14
    assert rel_l2(got, ref) <= 1e-12, rel_l2(got, ref)
    assert rel_l2(got, phit) <= 1e-12
    check_boundary(got, p)


@pytest.mark.parametrize("shape", [(3, 4, 3), (3, 5, 9), (9, 1, 3), (7, 2, 6), (10, 3, 11), (12, 5, 7),
                                   (18, 6, 20), (35, 9, 34)])
def test_solve_edge_shapes_match_dense(P, shape):
    """Single-level grids (Nr or Nz = 3), Ntheta in {1, 2}, odd Ntheta, odd interval counts
    (non-uniform coarse grids), against brute-force or sparse direct solves."""
    nr, nt, nz = shape
    p = W.HIGH_SHIFT.with_sizes(nr, nt, nz)
    rho = W.blob_charge(p, seed=nr * 7 + nt)
    g = fv.Grid.of(p)
    ref = solvers.solve_dense(g, rho, p.bc) if g.n_unknowns <= 3000 else solvers.solve_sparse(g, rho, p.bc)
    say("solve-edge", shape)
    plan = P.Plan.for_problem(p)
    phi, st = plan.solve(dev(rho), tol=1e-14)
    got = host(phi)
    assert st["status"] == P.OK, st
    assert rel_l2(got, ref) <= 1e-12, rel_l2(got, ref)
    check_boundary(got, p)


@pytest.mark.parametrize("prob", [W.BATCHED, W.HIGH_SHIFT])
def test_solve_matches_separable(P, prob):
    rho = W.blob_charge(prob, seed=24680)
    ref = solvers.solve_separable(fv.Grid.of(prob), rho, prob.bc)
    say("solve", prob.name)
    plan = P.Plan.for_problem(prob)
    phi, st = plan.solve(dev(rho), tol=1e-14)
    got = host(phi)
    assert st["status"] == P.OK, st
    assert rel_l2(got, ref) <= 1e-12, rel_l2(got, ref)
    check_boundary(got, prob)


def test_solve_planes_matches_mode_systems(P):
    """Each plane solves (A_0 + lambda_m M) u = b (Eq. shifted_operator_family), with its own
    Dirichlet ring, against the oracle's sparse solve of that 2-D system."""
    p = W.HIGH_SHIFT.with_sizes(19, 6, 14)
    g = fv.Grid.of(p)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(p.shape)
    ring = np.zeros(p.shape)
    ring[:, 0, :] = rng.standard_normal((p.ntheta, p.nr))
    ring[:, :, 0] = rng.standard_normal((p.ntheta, p.nz))
    lam = spectral.plane_eigenvalues(p.ntheta, float(g.dtheta))
    ref = np.empty(g.interior_shape)
    for q in range(p.ntheta):
        rhs_q = b[q][1:-1, 1:-1] + fv.rhs(g, np.zeros(g.shape), ring)[q]
        ref[q] = solvers.solve_mode(g, lam[q], rhs_q)
    say("solve_planes")
    plan = P.Plan.for_problem(p)
    u = dev(ring)
    P.solve_planes(plan.handle, dev(b), u, 1e-14)
    got = host(u)
    assert rel_l2(got[INTERIOR], ref, where=Ellipsis) <= 1e-12
    np.testing.assert_array_equal(got[:, 0, :], ring[:, 0, :])
    np.testing.assert_array_equal(got[:, :, 0], ring[:, :, 0])


def test_boundary_data_only_enters_plane_zero(P):
    """rho = 0: only m = 0 carries a boundary term (Eq. mode_rhs), so every other plane stays
    exactly zero and phi is exactly theta-invariant."""
    p = W.SMALL.with_sizes(21, 8, 17)
    say("rho=0")
    plan = P.Plan.for_problem(p)
    phi, st = plan.solve(torch.zeros(p.shape, dtype=torch.float64, device="cuda:0"), tol=1e-14)
    got = host(phi)
    assert (got == got[:1]).all()
    ref = solvers.solve_sparse(fv.Grid.of(p), np.zeros(p.shape), p.bc)
    assert rel_l2(got, ref) <= 1e-12
    assert got[INTERIOR].min() > 0 and got[INTERIOR].max() < 300


def test_theta_reflection(P):
    """theta -> -theta maps cos planes to themselves and negates sin planes; the solution reflects."""
    p = W.SMALL.with_sizes(17, 12, 17)
    rho = W.blob_charge(p, 9)
    refl = np.ascontiguousarray(rho[(-np.arange(p.ntheta)) % p.ntheta])
    say("reflection")
    plan = P.Plan.for_problem(p)
    a, _ = plan.solve(dev(rho), tol=1e-14)
    b, _ = plan.solve(dev(refl), tol=1e-14)
    a, b = host(a), host(b)
    assert rel_l2(b, a[(-np.arange(p.ntheta)) % p.ntheta]) <= 1e-13


# ------------------------------------------------------------- failures
def test_non_finite_rho_is_reported(P):
    p = W.SMALL.with_sizes(9, 4, 9)
    rho = W.blob_charge(p, 1)
    rho[2, 3, 4] = np.nan
    say("nan rho")
    plan = P.Plan.for_problem(p)
    phi = torch.full(p.shape, 7.0, dtype=torch.float64, device="cuda:0")
    with pytest.raises(P.CylPoissonError) as e:
        plan.solve(dev(rho), phi=phi)
    assert e.value.status == P.ENONFINITE
    assert (host(phi) == 7.0).all()


@pytest.mark.parametrize("shape", [(9, 4, 9), (129, 8, 129)])
def test_zero_problem_needs_no_cycle(P, shape):
    """rho = 0 with zero face values: the zero field solves it; no cycle is
    counted and the answer is exactly zero (the right-hand side's norm may come
    back only with the first cycles' norms, which must not change it)."""
    import dataclasses
    p = dataclasses.replace(W.SMALL.with_sizes(*shape), phi_zL=0.0)
    say("zero problem", shape)
    plan = P.Plan.for_problem(p)
    phi = torch.full(p.shape, 7.0, dtype=torch.float64, device="cuda:0")
    _, st = plan.solve(dev(np.zeros(p.shape)), tol=1e-12, phi=phi)
    assert st["status"] == P.OK and st["cycles"] == 0 and st["rel_residual"] == 0.0
    assert st["initial_residual_norm"] == 0.0
    assert (host(phi) == 0.0).all()


@pytest.mark.parametrize("shape", [(129, 8, 129)])
def test_non_finite_rho_is_reported_on_fused_grids(P, shape):
    p = W.SMALL.with_sizes(*shape)
    rho = W.blob_charge(p, 1)
    rho[5, 60, 70] = np.inf
    say("inf rho", shape)
    plan = P.Plan.for_problem(p)
    phi = torch.full(p.shape, 7.0, dtype=torch.float64, device="cuda:0")
    with pytest.raises(P.CylPoissonError) as e:
        plan.solve(dev(rho), phi=phi)
    assert e.value.status == P.ENONFINITE
    assert (host(phi) == 7.0).all()
    # the plan solves the next problem normally
    phi2, st = plan.solve(dev(W.blob_charge(p, 2)), tol=1e-12)
    assert st["status"] == P.OK and np.isfinite(host(phi2)).all()


def test_not_converged_returns_last_iterate(P):
    p = W.SMALL
    rho = W.blob_charge(p, 2)
    say("max_cycles=1")
    plan = P.Plan.for_problem(p, max_cycles=1)
    phi, st = plan.solve(dev(rho), tol=1e-14, allow=(P.OK, P.NOT_CONVERGED))
    assert st["status"] == P.NOT_CONVERGED and st["cycles"] == 1
    assert 1e-14 < st["rel_residual"] < 0.2
    check_boundary(host(phi), p)


def test_tolerance_below_the_floor_stops_on_stagnation(P):
    """A tolerance no FP64 iteration can reach: the cycles stop once the residual
    falls less than 0.6-fold over three checks, with NOT_CONVERGED, the
    stagnation message and an answer at the oracle's floor."""
    p = W.SMALL
    _, rho = manufactured(p)
    ref = solvers.solve_sparse(fv.Grid.of(p), rho, p.bc)
    say("stagnation tol 1e-22")
    plan = P.Plan.for_problem(p)
    phi, st = plan.solve(dev(rho), tol=1e-22, allow=(P.OK, P.NOT_CONVERGED))
    assert st["status"] == P.NOT_CONVERGED, st
    assert "stagnated" in P.last_error(), P.last_error()
    assert st["cycles"] < plan.get_option("max_cycles"), st
    assert st["rel_residual"] < 1e-14, st
    assert rel_l2(host(phi), ref) <= 1e-12
    check_boundary(host(phi), p)


def test_oversized_plan_reports_enomem_and_releases_its_memory(P):
    """A workspace larger than the device's memory (16001 x 256 x 16385 nodes:
    537 GB per node array) fails with ENOMEM, frees what it took, and a normal
    plan created after it still solves."""
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    say("oversized plan")
    with pytest.raises(P.CylPoissonError) as e:
        P.Plan(16001, 256, 16385, 0.02, 0.05, 0.05 / 16384, (0.0, 0.0, 0.0, 300.0))
    assert e.value.status == P.ENOMEM, (e.value.status, str(e.value))
    assert P.last_status() == P.ENOMEM
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] >= free0 - (64 << 20)
    p = W.SMALL
    _, rho = manufactured(p)
    phi, st = P.Plan.for_problem(p).solve(dev(rho), tol=1e-14)
    assert st["status"] == P.OK and P.last_status() == P.OK
    assert rel_l2(host(phi), solvers.solve_sparse(fv.Grid.of(p), rho, p.bc)) <= 1e-12


def test_host_pointer_is_rejected(P):
    p = W.SMALL.with_sizes(5, 2, 5)
    plan = P.Plan.for_problem(p)
    cpu = torch.zeros(p.shape, dtype=torch.float64)
    gpu = torch.zeros(p.shape, dtype=torch.float64, device="cuda:0")
    with pytest.raises(P.CylPoissonError) as e:
        P.solve(plan.handle, cpu, gpu)
    assert e.value.status == P.EDEVICE
    # the binding checks tensor shapes (the C ABI can only check allocation bounds)
    with pytest.raises(ValueError):
        plan.solve(torch.zeros(3, dtype=torch.float64, device="cuda:0"))


# ------------------------------------------------------------ full size
@pytest.mark.slow
def test_paper_scale_matches_separable_oracle(P):
    """400 x 128 x 512 (65 modes), manufactured rho: against the exact separable solver and phi_true."""
    p = W.PAPER_SCALE
    phit = W.manufactured_potential(p, 12345)
    say("paper-scale: forming rho on the CPU")
    phit_ld, rho = manufactured(p)
    ref = solvers.solve_separable(fv.Grid.of(p), rho, p.bc, workers=16)
    say("paper-scale solve")
    plan = P.Plan.for_problem(p)
    phi, st = plan.solve(dev(rho), tol=1e-14)
    got = host(phi)
    assert st["status"] == P.OK, st
    assert rel_l2(got, ref) <= 1e-12, rel_l2(got, ref)
    assert rel_l2(got, phit) <= 1e-12
    check_boundary(got, p)


# -------------------------------------------------- fused vs per-step path
@pytest.mark.parametrize("direct", [0, 1, 2])
@pytest.mark.parametrize("shape", [(33, 16, 33), (40, 8, 37), (129, 8, 129), (26, 3, 71), (129, 4, 33),
                                   (33, 4, 200), (257, 4, 129)])
def test_fused_passes_match_per_step_kernels(P, shape, direct):
    """The fused streaming passes run the same red-black schedule and point arithmetic as the
    one-kernel-per-step path (with contraction pinned in the shared point operations), so the
    iterates agree bitwise; with the exact coarse-level solve both paths stop there."""
    nr, nt, nz = shape
    p = W.SMALL.with_sizes(nr, nt, nz)
    rho = dev(W.blob_charge(p, seed=nr + nz))
    say("fused-vs-step", shape, "direct", direct)
    a = P.Plan.for_problem(p, fused=1, max_cycles=6, direct=direct)
    b = P.Plan.for_problem(p, fused=0, max_cycles=6, direct=direct)
    pa, sa = a.solve(rho, tol=1e-30, allow=(P.OK, P.NOT_CONVERGED))
    pb, sb = b.solve(rho, tol=1e-30, allow=(P.OK, P.NOT_CONVERGED))
    ha, hb = host(pa), host(pb)
    assert sa["cycles"] == sb["cycles"] == 6
    np.testing.assert_array_equal(ha, hb)
    # the residual norms are summed in another order (per chunk against per
    # workgroup of the norm kernel): they agree to rounding of the sums
    both = [(x, y) for x, y in zip(sa["history"][:6], sb["history"][:6]) if x is not None and y is not None]
    assert both
    np.testing.assert_allclose([x for x, _ in both], [y for _, y in both], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("chunk", [1, 5, 16, 1000])
def test_fused_chunking_is_exact(P, chunk):
    """Chunk boundaries (axial halos recomputed per workgroup) do not change the result."""
    p = W.SMALL.with_sizes(45, 8, 61)
    rho = dev(W.blob_charge(p, seed=4))
    say("chunk", chunk)
    ref_plan = P.Plan.for_problem(p, fused=0, max_cycles=3)
    r, _ = ref_plan.solve(rho, tol=1e-30, allow=(P.OK, P.NOT_CONVERGED))
    r = host(r).copy()
    plan = P.Plan.for_problem(p, chunk_rows=chunk, max_cycles=3)
    x, _ = plan.solve(rho, tol=1e-30, allow=(P.OK, P.NOT_CONVERGED))
    np.testing.assert_array_equal(host(x), r)


@pytest.mark.parametrize("pd", [2, 3])
def test_prefetch_depth_is_exact(P, pd):
    """Rows loaded further ahead change when values arrive, not what is computed."""
    p = W.SMALL.with_sizes(257, 8, 193)
    rho = dev(W.blob_charge(p, seed=pd))
    say("prefetch", pd)
    r, sr = P.Plan.for_problem(p, max_cycles=4).solve(rho, tol=1e-30, allow=(P.OK, P.NOT_CONVERGED))
    r = host(r).copy()
    x, sx = P.Plan.for_problem(p, prefetch=pd, max_cycles=4).solve(rho, tol=1e-30,
                                                                   allow=(P.OK, P.NOT_CONVERGED))
    np.testing.assert_array_equal(host(x), r)
    assert sx["history"] == sr["history"]


def test_prefetch_beyond_three_rows_is_rejected(P):
    plan = P.Plan.for_problem(W.SMALL)
    with pytest.raises(P.CylPoissonError):
        plan.set_option("prefetch", 4)
    assert plan.get_option("prefetch") == 1


@pytest.mark.parametrize("shape", [(129, 8, 129), (65, 5, 97), (401, 4, 65)])
def test_bottom_kernel_matches_level_by_level(P, shape):
    """The LDS bottom kernel (all small levels of a plane in one workgroup) runs the same
    V-cycle as the level-by-level kernels."""
    nr, nt, nz = shape
    p = W.SMALL.with_sizes(nr, nt, nz)
    rho = dev(W.blob_charge(p, seed=nt))
    say("bottom", shape)
    # the V-cycle must reach the bottom kernel's levels: no exact solve above them
    a = P.Plan.for_problem(p, bottom=1, max_cycles=4, direct=0)
    b = P.Plan.for_problem(p, bottom=0, max_cycles=4, direct=0)
    assert a.info()["bottom_level"] >= 1
    pa, sa = a.solve(rho, tol=1e-30, allow=(P.OK, P.NOT_CONVERGED))
    pa = host(pa).copy()
    pb, sb = b.solve(rho, tol=1e-30, allow=(P.OK, P.NOT_CONVERGED))
    # the same point operations in the same red-black order, and the same
    # coarsest product: bitwise
    np.testing.assert_array_equal(pa, host(pb))
    assert sa["history"] == sb["history"]


# ------------------------------------------------- plane groups on streams
@pytest.mark.parametrize("groups", [2, 3, 4])
@pytest.mark.parametrize("precision", [64, 32])
def test_plane_groups_are_bitwise_identical(P, groups, precision):
    """Each plane's arithmetic does not depend on how planes are grouped onto
    streams, so grouped solves reproduce the single-stream result exactly."""
    p = W.BATCHED.with_sizes(129, 24, 97)
    rho = dev(W.blob_charge(p, seed=11))
    say("plane groups", groups, "precision", precision)
    base = P.Plan.for_problem(p)
    grouped = P.Plan.for_problem(p, groups=groups)
    if precision == 32:
        base.set_option("precision", 32)
        grouped.set_option("precision", 32)
    a, sa = base.solve(rho, tol=1e-14)
    a = host(a).copy()
    b, sb = grouped.solve(rho, tol=1e-14)
    np.testing.assert_array_equal(a, host(b))
    assert sa["cycles"] == sb["cycles"] and histories_agree(sa["history"], sb["history"])


# ------------------------------------------------ anisotropic cells
@pytest.mark.parametrize("shape", [(129, 4, 33), (401, 8, 65), (33, 8, 257), (65, 16, 513)])
def test_anisotropic_grids_converge_and_match_the_oracle(P, shape):
    """Cells up to 10:1 (either way round): the hierarchy coarsens only the
    strongly coupled direction until the cells are within 2:1, so the point
    smoother keeps its multigrid rate."""
    p = W.SMALL.with_sizes(*shape)
    rho = W.blob_charge(p, seed=3)
    ref = solvers.solve_separable(fv.Grid.of(p), rho, p.bc)
    say("anisotropic", shape)
    phi, st = P.Plan.for_problem(p).solve(dev(rho), tol=1e-13)
    assert st["status"] == P.OK and st["cycles"] <= 14, st
    assert rel_l2(host(phi), ref) <= 1e-12


@pytest.mark.parametrize("nus", [(1, 1), (3, 2), (4, 4)])
@pytest.mark.parametrize("fused", [1, 0])
def test_coarse_sweep_counts_reach_the_oracle(P, nus, fused):
    """nu1_coarse / nu2_coarse change the sweeps below the finest level only (fused
    passes, per-step kernels and the LDS bottom kernel); the answer is the oracle's."""
    p = W.BATCHED.with_sizes(97, 8, 129)
    rho = W.blob_charge(p, seed=31)
    ref = solvers.solve_separable(fv.Grid.of(p), rho, p.bc)
    say("coarse sweeps", nus, "fused", fused)
    plan = P.Plan.for_problem(p, nu1_coarse=nus[0], nu2_coarse=nus[1], fused=fused)
    assert plan.get_option("nu1_coarse") == nus[0] and plan.get_option("nu2_coarse") == nus[1]
    phi, st = plan.solve(dev(rho), tol=1e-14)
    assert st["status"] == P.OK, st
    assert rel_l2(host(phi), ref) <= 1e-12, rel_l2(host(phi), ref)


# ------------------------------------------- merged finest pass (option merge)
@pytest.mark.parametrize("shape,options", [((400, 16, 512), {}), ((129, 8, 129), {}), ((201, 5, 97), {}),
                                           ((257, 8, 257), {"fmg": 1}), ((129, 8, 129), {"merge_prefetch": 2}),
                                           # 5 and 6 sweeps in one merged pass
                                           ((400, 16, 512), {"nu1": 3, "fmg": 1}), ((201, 5, 97), {"nu2": 3}),
                                           ((129, 8, 129), {"nu1": 3, "nu2": 3, "merge_prefetch": 2})],
                         ids=["400x16x512", "129x8x129", "201x5x97", "fmg-257", "prefetch2", "v32-fmg", "v23",
                              "v33-prefetch2"])
def test_merged_finest_passes_equal_the_separate_passes(P, shape, options):
    """A cycle without a check ends in one finest pass doing its up pass and the
    next cycle's down pass, with the node arithmetic of the two: iterates and
    answers are bitwise those of separate passes.  A fixed check schedule
    (tol 1e-30: checks after cycles 2 and 7) merges the boundaries after
    cycles 1, 3, 4, 5 and 6."""
    nr, nt, nz = shape
    p = W.SMALL.with_sizes(nr, nt, nz)
    rho = dev(W.blob_charge(p, seed=nr + nt))
    say("merged passes", shape, options)
    a = P.Plan.for_problem(p, merge=1, max_cycles=7, timing=1, **options)
    b = P.Plan.for_problem(p, merge=0, max_cycles=7, **options)
    pa, sa = a.solve(rho, tol=1e-30, allow=(P.OK, P.NOT_CONVERGED))
    pa = host(pa).copy()
    pb, sb = b.solve(rho, tol=1e-30, allow=(P.OK, P.NOT_CONVERGED))
    np.testing.assert_array_equal(pa, host(pb))
    assert sa["cycles"] == sb["cycles"] == 7
    assert sa["kernel_launches"]["fine_merged"] == 5, sa["kernel_launches"]
    assert [h is None for h in sa["history"]] == [True, False, True, True, True, True, False]
    assert histories_agree(sa["history"], sb["history"])


def test_timing_two_records_the_finest_passes_only(P):
    """Option timing = 2 brackets only the finest-level passes with events (the
    classes the roofline figures use); timing = 1 brackets every launch."""
    p = W.SMALL.with_sizes(65, 8, 65)
    rho = dev(W.blob_charge(p, seed=12))
    say("timing modes")
    plan = P.Plan.for_problem(p, timing=2)
    _, st = plan.solve(rho, tol=1e-13)
    kl = st["kernel_launches"]
    assert kl["fine_up"] >= 1 and kl["fine_down"] >= 1 and st["kernel_ms"]["fine_up"] > 0, kl
    assert kl["coarse_levels"] == kl["other"] == kl["dft_forward"] == kl["dft_inverse"] == 0, kl
    plan.set_option("timing", 1)
    _, st = plan.solve(rho, tol=1e-13)
    assert st["kernel_launches"]["coarse_levels"] >= 1 and st["kernel_launches"]["dft_forward"] == 1


def test_first_check_follows_the_last_converged_solve(P):
    """A repeated solve to the same tol checks first at the cycle count the last
    one needed: fewer host round trips, the same answer."""
    p = W.BATCHED
    rho = dev(W.blob_charge(p, seed=5))
    plan = P.Plan.for_problem(p, fmg=1)
    say("first check from history")
    a, sa = plan.solve(rho, tol=1e-13)
    a = host(a).copy()
    b, sb = plan.solve(rho, tol=1e-13)
    assert sa["status"] == sb["status"] == P.OK
    assert sb["cycles"] == sa["cycles"] and sb["checks"] < sa["checks"], (sa, sb)
    np.testing.assert_array_equal(a, host(b))
    # another tolerance, or a changed option, starts from the default schedule again
    _, sc = plan.solve(rho, tol=1e-12)
    assert sc["status"] == P.OK
    plan.set_option("nu1", 2)
    _, sd = plan.solve(rho, tol=1e-13)
    assert sd["checks"] == sa["checks"]


def test_warm_first_check_not_from_a_cold_solve(P):
    """Warm starts close to the answer predict their first check from the last
    warm solve's contraction factor, never from a solve that started far away:
    a small drift of the charge then needs fewer cycles than the solve from
    zero."""
    p = W.BATCHED
    rho = W.blob_charge(p, seed=5)
    drift = W.drift_fields(p, count=2, seed=11)
    amp = 1e-3 * float(np.abs(rho).max())
    plan = P.Plan.for_problem(p, warm_start=1)
    phi = dev(np.zeros(p.shape))
    say("warm first check")
    _, s0 = plan.solve(dev(rho), tol=1e-13, phi=phi)
    stats = []
    for k in range(8):
        rho = rho + amp * drift[k % 2]
        _, st = plan.solve(dev(rho), tol=1e-13, phi=phi)
        assert st["status"] == P.OK, st
        stats.append(st)
    assert all(st["cycles"] < s0["cycles"] for st in stats), (s0, stats)
    # the starting residual's read-back, then at most one check before the
    # predicted one (the factor varies a little from step to step)
    assert all(st["checks"] <= 3 for st in stats), stats
    # cycles between checks end in merged passes and form no norms: the first
    # formed norm is the first check, never later than the last solve's count
    # (a solve ending on the rounding floor must not push the next one on)
    for prev, st in zip(stats, stats[1:]):
        first = next(i for i, h in enumerate(st["history"]) if h is not None) + 1
        assert first <= prev["cycles"], (prev, st)
    ref = solvers.solve_separable(fv.Grid.of(p), rho, p.bc)
    assert rel_l2(host(phi), ref) < 1e-12


# ------------------------------------------- exact solve of a coarse level
@pytest.mark.parametrize("direct", [1, 2])
@pytest.mark.parametrize("prob,tol", [(W.SMALL, 1e-14), (W.BATCHED, 1e-14), (W.HIGH_SHIFT, 1e-14),
                                      # direct = 1 takes a level above 64 nodes each way
                                      # (two-kernel form): 128 x 128 (the largest), 127 x 127,
                                      # 99 x 127, 107 x 46 and 15 x 99 interior nodes
                                      (W.SMALL.with_sizes(259, 4, 259), 1e-14),
                                      (W.SMALL.with_sizes(257, 4, 257), 1e-14),
                                      (W.SMALL.with_sizes(400, 8, 512), 1e-14),
                                      (W.SMALL.with_sizes(217, 6, 94), 1e-14),
                                      (W.SMALL.with_sizes(65, 5, 401), 1e-14),
                                      # cells 20:1, coarsened in r only: the residual's FP64
                                      # floor is 5e-14 with or without the exact solve
                                      (W.SMALL.with_sizes(401, 4, 65), 1e-13)],
                         ids=lambda x: f"{x.nr}x{x.ntheta}x{x.nz}" if hasattr(x, "nr") else str(x))
def test_direct_coarse_solve_matches_oracle(P, prob, tol, direct):
    """The V-cycle stopping at a level solved exactly (axial eigenvectors, radial
    tridiagonal solves) meets the oracle, converges at least as fast per cycle as
    the V-cycle through every level (its coarse correction is exact rather than
    one V-cycle's), and contracts like a two- or three-grid method; in both
    forms (direct = 1: up to 128 interior nodes each way, direct = 2: up to 64)."""
    rho = W.blob_charge(prob, seed=prob.nz)
    ref = solvers.solve_separable(fv.Grid.of(prob), rho, prob.bc)
    say("direct", direct, prob.nr, prob.ntheta, prob.nz)
    a = P.Plan.for_problem(prob, direct=direct)
    b = P.Plan.for_problem(prob, direct=0)
    pa, sa = a.solve(dev(rho), tol=tol)
    pa = host(pa).copy()
    pb, sb = b.solve(dev(rho), tol=tol)
    assert sa["status"] == sb["status"] == P.OK, (sa, sb)
    if a.info()["direct_level"] < 1:
        # no level small enough at or above the bottom kernel's: the option is ignored
        np.testing.assert_array_equal(pa, host(pb))
        return
    assert rel_l2(pa, ref) <= 1e-12, rel_l2(pa, ref)
    assert rel_l2(host(pb), ref) <= 1e-12
    assert sa["cycles"] <= sb["cycles"], (sa["cycles"], sb["cycles"])

    def rate(st):
        # mean contraction per cycle from the first formed norm to the last
        h = [(i + 1, x) for i, x in enumerate(st["history"]) if x is not None]
        (c0, r0), (c1, r1) = h[0], h[-1]
        return (r1 / r0) ** (1.0 / (c1 - c0)) if c1 > c0 else 0.0

    # a broken coarse solve would leave the V-cycle contracting by 0.5 or worse
    assert rate(sa) < 0.1, sa["history"]


def test_direct_level_choice(P):
    """Option direct = 1 (the default) takes the first level from 1 on with at
    most 128 interior nodes each way, direct = 2 the first with at most 64 (one
    workgroup's LDS holds the plane and its transforms); with direct = 0 the
    V-cycle goes down to the bottom kernel."""
    info = P.Plan.for_problem(W.PAPER_SCALE).info()
    assert info["direct_level"] == 2, info  # (400, 512) -> (201, 257) -> (101, 129)
    shapes = info["level_shapes"]
    assert shapes[2][1] - 2 <= 128 < shapes[1][1] - 2 and shapes[2][0] - 2 <= 128
    info = P.Plan.for_problem(W.PAPER_SCALE, direct=2).info()
    assert info["direct_level"] == 3, info  # -> (51, 65)
    assert shapes[3][1] - 2 <= 64 < shapes[2][1] - 2 and shapes[3][0] - 2 <= 64
    assert P.Plan.for_problem(W.PAPER_SCALE, direct=0).info()["direct_level"] == -1
    # the option can change on a built plan
    plan = P.Plan.for_problem(W.SMALL.with_sizes(257, 4, 257))
    assert plan.info()["direct_level"] == 1
    plan.set_option("direct", 2)
    assert plan.info()["direct_level"] == 2
    info = P.Plan.for_problem(W.BATCHED).info()
    assert info["direct_level"] == 1, info
    plan = P.Plan.for_problem(W.BATCHED, direct=0)
    on = P.Plan.for_problem(W.BATCHED)
    assert on.get_option("direct") == 1  # on by default
    # the V-cycle stops at the direct level: no more levels run fused passes
    assert on.info()["fused_levels"] <= plan.info()["fused_levels"]
