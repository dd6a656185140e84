"""cylpoisson_solve_static: the solve with every V-cycle work array in the
library's static device scratch, for callers that cannot allocate.  It runs
the kernels of cylpoisson_solve on other buffers, so its answer and residual
history equal the plan-workspace solve's bit for bit; checked on two calls in
a row, the second on a smaller grid (the scratch keeps the first call's
contents), plus the oracle and the size and option limits."""
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
    return P


@pytest.mark.parametrize("fmg", [0, 1])
def test_static_scratch_solve_equals_the_plan_solve(P, fmg):
    # the largest grid of the first call fills most of the 64 MiB scratch
    for p, seed in ((W.BATCHED, 24680), (W.SMALL.with_sizes(65, 16, 97), 7)):
        rho = W.blob_charge(p, seed)
        ref = solvers.solve_separable(fv.Grid.of(p), rho, p.bc)
        plan = P.Plan.for_problem(p, fmg=fmg)
        r = dev(rho)
        say("static scratch", p.shape, "fmg", fmg)
        a, sa = plan.solve(r, tol=1e-13)
        a = host(a).copy()
        b, sb = plan.solve_static(r, tol=1e-13)
        b = host(b)
        assert sa["status"] == P.OK and sb["status"] == P.OK, (sa, sb)
        assert sa["cycles"] == sb["cycles"] and histories_agree(sa["history"], sb["history"])
        np.testing.assert_array_equal(a, b)
        assert rel_l2(b, ref) <= 1e-12
        # the plan's own solve still works after the static one
        c, _ = plan.solve(r, tol=1e-13)
        np.testing.assert_array_equal(host(c), a)
        plan.close()


def test_static_scratch_limits(P):
    too_big = P.Plan.for_problem(W.BATCHED.with_sizes(257, 64, 129))
    r = torch.zeros(too_big.shape, dtype=torch.float64, device="cuda:0")
    say("static scratch limits")
    with pytest.raises(P.CylPoissonError) as e:
        too_big.solve_static(r)
    assert e.value.status == P.EINVAL and "static scratch" in P.last_error()
    small = P.Plan.for_problem(W.SMALL, precision=32)
    r = torch.zeros(small.shape, dtype=torch.float64, device="cuda:0")
    with pytest.raises(P.CylPoissonError) as e:
        small.solve_static(r)
    assert e.value.status == P.EINVAL
    # a problem whose answer is zero (no charge, grounded faces) needs no cycle
    zero = P.Plan.for_problem(dataclasses.replace(W.SMALL, phi_zL=0.0))
    phi, st = zero.solve_static(r, tol=1e-12)
    assert st["status"] == P.OK and st["cycles"] == 0 and (host(phi) == 0).all()
