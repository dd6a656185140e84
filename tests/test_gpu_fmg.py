"""The full-multigrid start (option "fmg"): the right-hand side restricted to
the level where the V-cycle stops, solved there (exactly, or by the bottom
kernel from zero), one V-cycle per level on the way up
from the interpolated coarser answer, then V-cycles on the finest level from
the interpolated level-1 answer.  It changes the starting iterate only, so the
solve must still meet the oracle, take no more cycles than the zero start, and
give bitwise the same answer under plane groups and graph replay."""
import dataclasses

import numpy as np
import pytest
import torch

import workloads as W
from oracle import fv, solvers

from gpu_util import dev, histories_agree, host, rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2609_07172_amd as P
    P.library()
    assert torch.cuda.is_available()
    return P


@pytest.mark.parametrize("prob", [W.SMALL.with_sizes(257, 8, 257), W.BATCHED, W.HIGH_SHIFT,
                                  W.SMALL.with_sizes(401, 4, 513),
                                  # uneven shapes: odd counts, other bottom levels and coarsenings
                                  W.SMALL.with_sizes(217, 6, 94), W.SMALL.with_sizes(105, 5, 344),
                                  W.SMALL.with_sizes(384, 4, 411), W.SMALL.with_sizes(76, 7, 259)],
                         ids=lambda p: f"{p.nr}x{p.ntheta}x{p.nz}")
@pytest.mark.parametrize("direct", [1, 2, 0])
def test_fmg_solve_matches_oracle(P, prob, direct):
    rho = W.blob_charge(prob, seed=prob.nr)
    ref = solvers.solve_separable(fv.Grid.of(prob), rho, prob.bc)
    say("fmg", prob.nr, prob.ntheta, prob.nz, "direct", direct)
    zero = P.Plan.for_problem(prob, direct=direct)
    plan = P.Plan.for_problem(prob, fmg=1, direct=direct)
    _, s0 = zero.solve(dev(rho), tol=1e-14)
    phi, st = plan.solve(dev(rho), tol=1e-14)
    got = host(phi)
    assert st["status"] == P.OK, st
    assert rel_l2(got, ref) <= 1e-12, rel_l2(got, ref)
    assert st["cycles"] <= s0["cycles"], (st["cycles"], s0["cycles"])
    np.testing.assert_array_equal(got[:, 0, :], prob.phi_z0)
    np.testing.assert_array_equal(got[:, -1, :], prob.phi_zL)


def test_fmg_on_a_stretched_cell_mesh(P):
    r = W.stretched_points(0.02, 0.05, 257, 1.004)
    z = W.stretched_points(0.0, 0.06, 300, 0.997)
    g = fv.Grid.cell_centred(r, z, 8)
    bc = (5.0, -3.0, 1.0, 300.0)
    rho = W.mesh_blob_charge(g.r, g.z, 8, seed=3)
    ref = solvers.solve_modes(g, rho, bc)
    say("fmg mesh", g.shape)
    plan = P.Plan.from_mesh(r, z, 8, P.CELL, bc, fmg=1)
    phi, st = plan.solve(dev(rho), tol=1e-13)
    assert st["status"] == P.OK, st
    assert rel_l2(host(phi), ref) <= 1e-12


@pytest.mark.parametrize("options", [dict(groups=3), dict(graph=1)], ids=["groups", "graph"])
def test_fmg_is_bitwise_under_groups_and_graphs(P, options):
    p = W.SMALL.with_sizes(257, 9, 257)
    rho = dev(W.blob_charge(p, seed=9))
    say("fmg", options)
    a, sa = P.Plan.for_problem(p, fmg=1).solve(rho, tol=1e-14)
    a = host(a).copy()
    plan = P.Plan.for_problem(p, fmg=1, **options)
    for _ in range(3):  # graph replays after the first capture
        b, sb = plan.solve(rho, tol=1e-14)
        np.testing.assert_array_equal(host(b), a)
        assert histories_agree(sb["history"], sa["history"])


def test_fmg_zero_problem_needs_no_cycle(P):
    p = dataclasses.replace(W.SMALL.with_sizes(257, 4, 257), phi_zL=0.0)
    say("fmg zero problem")
    plan = P.Plan.for_problem(p, fmg=1)
    phi = torch.full(p.shape, 7.0, dtype=torch.float64, device="cuda:0")
    _, st = plan.solve(dev(np.zeros(p.shape)), tol=1e-12, phi=phi)
    assert st["status"] == P.OK and st["cycles"] == 0
    assert (host(phi) == 0.0).all()


def test_fmg_with_masks_meets_the_oracle(P):
    """Planes frozen at the first check keep their full-multigrid iterate."""
    p = W.SMALL.with_sizes(257, 16, 257)
    rho = W.blob_charge(p, seed=12)
    ref = solvers.solve_separable(fv.Grid.of(p), rho, p.bc)
    say("fmg masks")
    plan = P.Plan.for_problem(p, fmg=1, masks=1)
    phi, st = plan.solve(dev(rho), tol=1e-13)
    assert st["status"] == P.OK, st
    assert rel_l2(host(phi), ref) <= 1e-12


def test_fmg_option_range(P):
    plan = P.Plan.for_problem(W.SMALL)
    for bad in (-1, 2, 0.5):
        with pytest.raises(P.CylPoissonError):
            plan.set_option("fmg", bad)
    plan.set_option("fmg", 1)
    assert plan.get_option("fmg") == 1


def test_fmg_fused_interpolation_is_exact(P):
    """With one row of prefetch the first finest down pass forms its start as
    it streams; with two it reads it from a written copy.  Prefetch changes no
    arithmetic, so the two solves agree bitwise."""
    p = W.SMALL.with_sizes(401, 5, 513)
    rho = dev(W.blob_charge(p, seed=21))
    say("fmg fused interpolation")
    a, sa = P.Plan.for_problem(p, fmg=1).solve(rho, tol=1e-14)
    a = host(a).copy()
    b, sb = P.Plan.for_problem(p, fmg=1, prefetch=2).solve(rho, tol=1e-14)
    np.testing.assert_array_equal(host(b), a)
    assert sa["history"] == sb["history"]
