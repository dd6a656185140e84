"""Warm starts, per-plane convergence masks, captured graphs, the launch-shape
autotuner and batched solves of uneven problems: each against the CPU oracle
(relative L2 <= 1e-12) or, where the arithmetic is the same, bitwise against
the plain solve.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fv, solvers

from gpu_util import INTERIOR as INNER, dev, histories_agree, host, rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2609_07172_amd as P
    P.library()
    assert torch.cuda.is_available()
    return P


def manufactured(p, seed=12345):
    phit = W.manufactured_potential(p, seed, np.longdouble)
    rho = fv.charge_from_potential(fv.Grid.of(p, np.longdouble), phit).astype(np.float64)
    return phit.astype(np.float64), rho


# ------------------------------------------------------------ warm starts
@pytest.mark.parametrize("precision", [64, 32])
def test_warm_start_from_the_solution_needs_no_cycle(P, precision):
    p = W.BATCHED.with_sizes(65, 16, 65)
    rho = dev(W.blob_charge(p, seed=5))
    plan = P.Plan.for_problem(p)
    if precision == 32:
        plan.set_option("precision", 32)
    phi, st = plan.solve(rho, tol=1e-13)
    ref = host(phi).copy()
    plan.set_option("warm_start", 1)
    phi2, st2 = plan.solve(rho, tol=1e-13, phi=phi)
    assert st2["status"] == P.OK and st2["cycles"] == 0, st2
    assert rel_l2(host(phi2), ref) <= 1e-14


@pytest.mark.parametrize("precision", [64, 32])
def test_warm_start_after_a_drift_is_faster_and_exact(P, precision):
    """A 1 % change of rho, started from the previous answer: fewer cycles than
    from zero, the same oracle answer (boundary nodes of the guess are garbage)."""
    p = W.BATCHED
    rho0 = W.blob_charge(p, seed=24680)
    rho1 = rho0 + 0.01 * np.abs(rho0).max() * W.blob_charge(p, seed=97531) / np.abs(
        W.blob_charge(p, seed=97531)).max()
    ref = solvers.solve_separable(fv.Grid.of(p), rho1, p.bc)
    say("warm start", precision)
    cold = P.Plan.for_problem(p)
    warm = P.Plan.for_problem(p, warm_start=0)
    if precision == 32:
        cold.set_option("precision", 32)
        warm.set_option("precision", 32)
    phi, _ = warm.solve(dev(rho0), tol=1e-14)
    g = host(phi).copy()
    g[:, 0, :] = 1e6  # the guess's boundary nodes must be ignored
    g[:, :, -1] = -7.0
    guess = dev(g)
    warm.set_option("warm_start", 1)
    phiw, sw = warm.solve(dev(rho1), tol=1e-14, phi=guess)
    phic, sc = cold.solve(dev(rho1), tol=1e-14)
    assert sw["status"] == P.OK and sw["cycles"] < sc["cycles"], (sw["cycles"], sc["cycles"])
    assert rel_l2(host(phiw), ref) <= 1e-12
    got = host(phiw)
    np.testing.assert_array_equal(got[:, 0, :], p.phi_z0)
    np.testing.assert_array_equal(got[:, 1:-1, -1], p.phi_r_out)


# -------------------------------------------------------------- masks
def test_masks_freeze_empty_planes_and_match_the_oracle(P):
    """The manufactured potential has harmonics m <= 3 only: every other plane
    has a right-hand side at rounding level and is frozen from the start."""
    p = W.SMALL.with_sizes(65, 32, 65)
    phit, rho = manufactured(p)
    ref = solvers.solve_sparse(fv.Grid.of(p), rho, p.bc) if False else solvers.solve_separable(
        fv.Grid.of(p), rho, p.bc)
    plan = P.Plan.for_problem(p, masks=1)
    phi, st = plan.solve(dev(rho), tol=1e-14)
    assert st["status"] == P.OK, st
    assert st["frozen_planes"] >= 32 - 7, st
    assert rel_l2(host(phi), ref) <= 1e-12


def test_masks_on_a_full_spectrum_match_the_oracle(P):
    p = W.BATCHED
    rho = W.blob_charge(p, seed=24680)
    ref = solvers.solve_separable(fv.Grid.of(p), rho, p.bc)
    phi, st = P.Plan.for_problem(p, masks=1).solve(dev(rho), tol=1e-14)
    assert st["status"] == P.OK and st["rel_residual"] <= 1e-14, st
    assert rel_l2(host(phi), ref) <= 1e-12


@pytest.mark.parametrize("fmg", [0, 1])
def test_masks_after_another_solve_keep_no_stale_plane(P, fmg):
    """A masked plan solves a full-spectrum charge, then the m <= 3 manufactured
    charge: the planes whose right-hand side is at rounding level now must hold
    this solve's answer, not the interior the previous solve left behind."""
    p = W.SMALL.with_sizes(129, 32, 129)
    phit, rho = manufactured(p)
    ref = solvers.solve_separable(fv.Grid.of(p), rho, p.bc)
    say("masks stale planes, fmg", fmg)
    plan = P.Plan.for_problem(p, masks=1, fmg=fmg)
    _, st0 = plan.solve(dev(W.blob_charge(p, seed=3)), tol=1e-14)
    assert st0["status"] == P.OK, st0
    phi, st = plan.solve(dev(rho), tol=1e-14)
    assert st["status"] == P.OK and st["frozen_planes"] >= 32 - 7, st
    got = host(phi)
    assert rel_l2(got, ref) <= 1e-12
    # planes m >= 4 carry rounding only: phi's azimuthal spectrum above m = 3
    # is at the oracle's level, not that of the blob charge's answer
    spec = np.abs(np.fft.rfft(got[INNER] - ref[INNER], axis=0)).max()
    assert spec <= 1e-10 * np.abs(ref).max(), spec


@pytest.mark.parametrize("options", [{}, {"fmg": 1}, {"masks": 1}, {"fmg": 1, "masks": 1}],
                         ids=["zero", "fmg", "masks", "fmg+masks"])
def test_tolerance_above_one_returns_the_zero_interior(P, options):
    """tol >= 1 is met by the zero interior before any cycle: the answer is that
    iterate (Dirichlet values on the boundary nodes, zero inside), whatever the
    plan's previous solve left in its buffers."""
    p = W.SMALL.with_sizes(129, 8, 129)
    plan = P.Plan.for_problem(p, **options)
    say("tol >= 1", options)
    plan.solve(dev(W.blob_charge(p, seed=3)), tol=1e-13)
    phi, st = plan.solve(dev(W.blob_charge(p, seed=4)), tol=1.0)
    assert st["status"] == P.OK and st["cycles"] == 0, st
    got = host(phi)
    assert (got[INNER] == 0.0).all()
    np.testing.assert_array_equal(got[:, 0, :], p.phi_z0)
    np.testing.assert_array_equal(got[:, -1, :], p.phi_zL)
    np.testing.assert_array_equal(got[:, 1:-1, 0], p.phi_r_in)
    np.testing.assert_array_equal(got[:, 1:-1, -1], p.phi_r_out)


# -------------------------------------------------------------- graphs
@pytest.mark.parametrize("options", [dict(fused=0), dict(smoother=2)], ids=["per-step", "lines"])
def test_graph_replays_on_the_per_step_path(P, options):
    """The one-kernel-per-step V-cycle (and the line smoothers on it) is captured
    and replayed too, bitwise equal to eager launches on every replay."""
    p = W.SMALL.with_sizes(65, 8, 49)
    eager = P.Plan.for_problem(p, **options)
    graph = P.Plan.for_problem(p, graph=1, **options)
    say("graph per-step", options)
    for seed in (1, 2, 3):
        r = dev(W.blob_charge(p, seed=seed))
        a, sa = eager.solve(r, tol=1e-13)
        b, sb = graph.solve(r, tol=1e-13)
        assert sa["cycles"] == sb["cycles"] and sb["status"] == P.OK
        np.testing.assert_array_equal(host(a), host(b))


@pytest.mark.parametrize("options", [{}, {"masks": 1}, {"fmg": 1, "masks": 1}], ids=["plain", "masks", "fmg-masks"])
def test_graph_replays_equal_eager_launches(P, options):
    """The cycles between two checks are captured on the first solve that runs
    them and replayed on later ones; every replay (with eager work and
    synchronisations in between) must give the eager result bit for bit, with
    per-plane masks updated between the segments too."""
    p = W.BATCHED.with_sizes(129, 16, 97)
    rhos = [dev(W.blob_charge(p, seed=s)) for s in (1, 2, 3)]
    eager = P.Plan.for_problem(p, **options)
    graph = P.Plan.for_problem(p, graph=1, **options)
    for rep in range(3):
        for r in rhos:
            a, sa = eager.solve(r, tol=1e-14)
            a = host(a).copy()
            torch.cuda.synchronize()
            b, sb = graph.solve(r, tol=1e-14)
            np.testing.assert_array_equal(a, host(b))
            assert histories_agree(sa["history"], sb["history"])


# ------------------------------------------------------------- autotune
def test_autotune_picks_candidates_and_keeps_results(P):
    p = W.BATCHED
    rho = W.blob_charge(p, seed=24680)
    ref = solvers.solve_separable(fv.Grid.of(p), rho, p.bc)
    plan = P.Plan.for_problem(p, omega=1.15, max_cycles=30)
    say("autotune", p.name)
    plan.autotune()
    assert plan.get_option("chunk_rows") in (0, 32, 48, 64, 96, 128)
    assert plan.get_option("chunk_rows_coarse") in (0, 16, 24, 32, 48, 64)
    assert plan.get_option("prefetch") in (1, 2, 3)
    assert plan.get_option("groups") in (1, 2, 4)
    assert plan.get_option("max_cycles") == 30 and plan.get_option("omega") == 1.15
    phi, st = plan.solve(dev(rho), tol=1e-14)
    assert rel_l2(host(phi), ref) <= 1e-12


# ---------------------------------------------------------------- batch
def test_batch_of_uneven_problems_matches_each_oracle(P):
    probs = [W.SMALL.with_sizes(nr, nt, nz) for nr, nt, nz in
             [(65, 32, 97), (33, 16, 33), (97, 8, 65), (40, 12, 71), (129, 4, 33), (17, 64, 129)]]
    rhos = [W.blob_charge(q, seed=100 + i) for i, q in enumerate(probs)]
    plans = [P.Plan.for_problem(q) for q in probs]
    say("batch of", len(probs))
    phis, sts = P.solve_plans(plans, [dev(r) for r in rhos], tol=1e-13)
    for q, r, phi, st in zip(probs, rhos, phis, sts):
        ref = solvers.solve_separable(fv.Grid.of(q), r, q.bc)
        assert st["status"] == P.OK, st
        assert rel_l2(host(phi), ref) <= 1e-12, q.shape
    # the same plans alone give the same bits
    for plan, r, phi in zip(plans, rhos, phis):
        alone, _ = plan.solve(dev(r), tol=1e-13)
        np.testing.assert_array_equal(host(alone), host(phi))


@pytest.mark.skip(reason="the shared-launch batch (one launch per pass over all problems) aborted the process in its first GPU run; the cause was not found and the path was taken out")
@pytest.mark.parametrize("fmg", [0, 1])
def test_lockstep_batch_is_bitwise_the_lone_solves(P, fmg):
    """The batch's V-cycles run in shared launches (one per pass over all
    problems; uneven widths, depths and bottom levels): every problem runs the
    cycles it would alone, with the same node arithmetic, so its answer, cycle
    count and checked residuals are those of its lone solve, and of the batch
    on separate streams."""
    probs = [W.SMALL.with_sizes(nr, nt, nz) for nr, nt, nz in
             [(65, 32, 97), (33, 16, 33), (97, 8, 65), (40, 12, 71), (257, 8, 129), (17, 64, 129), (129, 3, 257)]]
    rhos = [dev(W.blob_charge(q, seed=300 + i)) for i, q in enumerate(probs)]
    say("lockstep batch, fmg", fmg)
    lock = [P.Plan.for_problem(q, fmg=fmg, batch_lockstep=1) for q in probs]
    streams = [P.Plan.for_problem(q, fmg=fmg, batch_lockstep=0) for q in probs]
    alone = [P.Plan.for_problem(q, fmg=fmg) for q in probs]
    for rep in range(2):  # the second batch checks first where the first one converged
        a, sa = P.solve_plans(lock, rhos, tol=1e-14)
        a = [host(x).copy() for x in a]
        b, sb = P.solve_plans(streams, rhos, tol=1e-14)
        # cells more than 2:1 coarsen one direction only and run some levels on
        # per-step kernels: those problems run on streams of their own
        assert sum(x["lockstep"] for x in sa) >= 4, [x["lockstep"] for x in sa]
        assert not any(x["lockstep"] for x in sb)
        for i, (plan, r) in enumerate(zip(alone, rhos)):
            c, sc = plan.solve(r, tol=1e-14)
            np.testing.assert_array_equal(a[i], host(c))
            np.testing.assert_array_equal(a[i], host(b[i]))
            assert sa[i]["status"] == sc["status"] == P.OK
            assert sa[i]["cycles"] == sc["cycles"] == sb[i]["cycles"], (i, sa[i], sc)
            assert histories_agree(sa[i]["history"], sc["history"])
            ref = solvers.solve_separable(fv.Grid.of(probs[i]), W.blob_charge(probs[i], seed=300 + i),
                                          probs[i].bc) if rep == 0 else None
            if ref is not None:
                assert rel_l2(a[i], ref) <= 1e-12


@pytest.mark.skip(reason="the shared-launch batch (one launch per pass over all problems) aborted the process in its first GPU run; the cause was not found and the path was taken out")
def test_lockstep_batch_with_a_zero_problem_and_a_cycle_limit(P):
    """Problems that end at once (zero right-hand side, grounded boundary) or
    at their cycle limit leave the shared launches while the others go on."""
    import dataclasses
    grounded = dataclasses.replace(W.SMALL.with_sizes(65, 8, 65), phi_zL=0.0)
    probs = [W.BATCHED, grounded, W.SMALL.with_sizes(97, 4, 129)]
    rhos = [dev(W.blob_charge(W.BATCHED, seed=7)), torch.zeros(grounded.shape, dtype=torch.float64, device="cuda"),
            dev(W.blob_charge(probs[2], seed=8))]
    plans = [P.Plan.for_problem(probs[0], batch_lockstep=1), P.Plan.for_problem(probs[1], batch_lockstep=1),
             P.Plan.for_problem(probs[2], max_cycles=2, batch_lockstep=1)]
    say("lockstep batch with a zero problem")
    phis = [torch.full_like(r, 7.0) for r in rhos]
    status, sts = P.solve_batch([p.handle for p in plans], rhos, phis, tol=1e-13, allow=(P.OK, P.NOT_CONVERGED))
    assert status == P.NOT_CONVERGED and sts == [P.OK, P.OK, P.NOT_CONVERGED], sts
    assert all(p.stats()["lockstep"] == 1 for p in plans)
    assert plans[1].stats()["cycles"] == 0 and plans[2].stats()["cycles"] == 2
    assert float(phis[1].abs().max()) == 0.0
    ref = solvers.solve_separable(fv.Grid.of(W.BATCHED), W.blob_charge(W.BATCHED, seed=7), W.BATCHED.bc)
    assert rel_l2(host(phis[0]), ref) <= 1e-12
    alone, _ = P.Plan.for_problem(probs[2], max_cycles=2).solve(rhos[2], tol=1e-13, allow=(P.OK, P.NOT_CONVERGED))
    np.testing.assert_array_equal(host(alone), host(phis[2]))


def test_batch_reports_each_status(P):
    p = W.SMALL
    rho = dev(W.blob_charge(p, seed=1))
    a = P.Plan.for_problem(p)
    b = P.Plan.for_problem(p, max_cycles=1)
    status, sts = P.solve_batch([a.handle, b.handle], [rho, rho], [torch.empty_like(rho), torch.empty_like(rho)],
                                tol=1e-14, allow=(P.OK, P.NOT_CONVERGED))
    assert status == P.NOT_CONVERGED and sts == [P.OK, P.NOT_CONVERGED]
    with pytest.raises(P.CylPoissonError):
        P.solve_batch([a.handle, a.handle], [rho, rho], [torch.empty_like(rho), torch.empty_like(rho)])
