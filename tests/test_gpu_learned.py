"""The learned preconditioner: the network's BF16 matrix-core kernels against
the CPU oracle (forward, back-propagated gradients, Adam), training on
pairs from the plain solver (residuals of its V-cycle iterates and the
corrections its SOR smoother makes from them), and the learned solve, which is
judged against the plain V-cycle and must still reach the oracle's answer.

Tolerances: GPU and oracle round the same operands to BF16; the GPU keeps
activations in FP32 between layers, the oracle in FP64, so an activation
within FP32 rounding of a BF16 tie can round to the neighbouring BF16 value
(about 1 in 4e4 entries, each off by 2^-8 relative): relative L2 errors of
order 1e-5 on outputs and 1e-4 on gradients.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fv, nn, solvers

from gpu_util import dev, host, rel_l2, say

pytestmark = pytest.mark.gpu

RNG = np.random.Generator(np.random.PCG64(11))


@pytest.fixture(scope="module")
def P():
    import paper_2609_07172_amd as P
    P.library()
    assert torch.cuda.is_available()
    return P


def flat(params):
    return np.concatenate([p.astype(np.float32).ravel() for p in params])


def unflat(w):
    out, o = [], 0
    for ci, co in nn.SHAPES:
        n = 9 * ci * co
        out.append(w[o:o + n].astype(np.float64).reshape(9, ci, co))
        o += n
    return out


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def f32(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to("cuda:0")


@pytest.mark.parametrize("shape", [(2, 16, 16), (3, 20, 37), (1, 9, 70), (1, 1, 1), (2, 5, 3), (1, 17, 65),
                                   (2, 33, 129), (1, 48, 200)])
def test_forward_matches_oracle(P, shape):
    """The fused inference kernel (16 x 64 output tiles, halos in LDS): one
    pixel, tiles cut by the image edges, several tiles each way."""
    B, H, Wd = shape
    params = nn.init_params(5)
    net = P.Net(seed=1)
    net.set_weights(flat(params))
    x = RNG.standard_normal((B, H, Wd, 4)).astype(np.float32)
    y = net.forward(f32(x)).cpu().numpy()
    ref, _ = nn.forward(unflat(flat(params)), x.astype(np.float64), rounding=True)
    assert rel(y, ref) <= 1e-4, rel(y, ref)


def test_gradients_match_oracle(P):
    params = unflat(flat(nn.init_params(6)))
    net = P.Net(seed=1)
    net.set_weights(flat(params))
    x = RNG.standard_normal((3, 24, 40, 4)).astype(np.float32)
    t = RNG.standard_normal((3, 24, 40, 2)).astype(np.float32)
    loss = net.loss_grad(f32(x), f32(t))
    ref_loss, ref_grads = nn.loss_and_grads(params, x.astype(np.float64), t.astype(np.float64), rounding=True)
    assert loss == pytest.approx(ref_loss, rel=1e-4)
    g = unflat(net.get_grads())
    for l in range(3):
        assert rel(g[l], ref_grads[l]) <= 5e-4, (l, rel(g[l], ref_grads[l]))


def test_adam_step_matches_oracle(P):
    params = unflat(flat(nn.init_params(7)))
    net = P.Net(seed=1)
    net.set_weights(flat(params))
    x = RNG.standard_normal((2, 16, 32, 4)).astype(np.float32)
    t = RNG.standard_normal((2, 16, 32, 2)).astype(np.float32)
    net.loss_grad(f32(x), f32(t))
    grads = unflat(net.get_grads())
    net.adam_step(1e-2)
    state = [(np.zeros_like(p), np.zeros_like(p)) for p in params]
    ref = nn.adam_step(params, grads, state, lr=1e-2, step=1)
    got = unflat(net.get_weights())
    for l in range(3):
        np.testing.assert_allclose(got[l], ref[l], rtol=1e-5, atol=1e-6)


def test_training_on_solver_pairs_lowers_the_loss(P):
    p = W.SMALL.with_sizes(65, 16, 65)
    plan = P.Plan.for_problem(p)
    net = P.Net(seed=3)
    for k in range(2):
        rho = dev(W.blob_charge(p, seed=40 + k))
        net.collect(plan, rho, cycles=4, patches_per_cycle=64, seed=7 + k)
    assert net.patch_count() == 2 * 4 * 64
    say("training")
    first = net.train(epochs=1, batch=64, lr=2e-3)
    last = net.train(epochs=8, batch=64, lr=2e-3)
    assert last < 0.8 * first, (first, last)


@pytest.fixture(scope="module")
def trained(P):
    """A network trained on the residual/smoother-correction pairs of a 129 x 16 x 129 grid."""
    p = W.SMALL.with_sizes(129, 16, 129)
    plan = P.Plan.for_problem(p)
    net = P.Net(seed=5)
    for k in range(6):
        net.collect(plan, dev(W.blob_charge(p, seed=60 + k)), cycles=5, patches_per_cycle=128, seed=k)
    net.train(epochs=40, batch=128, lr=2e-3)
    net.train(epochs=20, batch=128, lr=5e-4)
    return p, net


def test_learned_solve_reaches_the_oracle(P, trained):
    p, net = trained
    rho = W.blob_charge(p, seed=99)
    ref = solvers.solve_separable(fv.Grid.of(p), rho, p.bc)
    plan = P.Plan.for_problem(p, krylov=1)
    P.plan_set_net(plan, net)
    phi, st = plan.solve(dev(rho), tol=1e-13)
    assert st["status"] == P.OK, st
    assert st["krylov_iterations"] >= 1 and st["vcycle_rate"] > 0 and st["learned_rate"] > 0
    assert rel_l2(host(phi), ref) <= 1e-12


def test_trained_network_beats_no_preconditioner(P, trained):
    """What the trained network gains over FGMRES without it (and over the
    untrained network): a smaller residual per FGMRES step over one restart.
    The smoother it imitates is printed beside it (measured: none 0.78, net
    0.73, four SOR sweeps 0.62, one V-cycle 0.053 per step at this size)."""
    p, net = trained
    rho = dev(W.blob_charge(p, seed=123))
    rates = {}
    for label, precond, n in (("none", 0, None), ("smoother", 2, None), ("untrained", 1, P.Net(seed=77)),
                              ("trained", 1, net)):
        plan = P.Plan.for_problem(p, krylov=1, krylov_precond=precond, fallback=0, krylov_max=8)
        if n is not None:
            P.plan_set_net(plan, n)
        _, st = plan.solve(rho, tol=1e-13, allow=(P.OK, P.NOT_CONVERGED))
        rates[label] = st["learned_rate"]
        say(label, st["learned_rate"], "v-cycle", st["vcycle_rate"])
    assert rates["trained"] < rates["none"], rates
    assert rates["trained"] < rates["untrained"], rates


def test_learned_solve_falls_back_when_worse(P, trained):
    """The network contracts far less per step than a V-cycle here: the judged
    solve hands over to V-cycles and still converges."""
    p, net = trained
    rho = W.blob_charge(p, seed=5)
    ref = solvers.solve_separable(fv.Grid.of(p), rho, p.bc)
    plan = P.Plan.for_problem(p, krylov=1)
    P.plan_set_net(plan, net)
    phi, st = plan.solve(dev(rho), tol=1e-13)
    if st["learned_rate"] >= st["vcycle_rate"]:
        assert st["learned_fallback"] == 1 and st["cycles"] >= 2
    assert st["status"] == P.OK and rel_l2(host(phi), ref) <= 1e-12


# ------------------- the network inside the V-cycle (krylov_precond 4)
@pytest.fixture(scope="module")
def trained_vcycle(P):
    """A network trained on 15,360 residual/smoother-correction pairs of the
    129 x 64 x 129 grid (five charges, six V-cycle iterates each)."""
    p = W.BATCHED
    plan = P.Plan.for_problem(p)
    net = P.Net(seed=2024)
    for k in range(5):
        net.collect(plan, dev(W.blob_charge(p, seed=100 + k)), cycles=6, patches_per_cycle=512, seed=k)
    net.train(epochs=30, batch=256, lr=2e-3)
    net.train(epochs=10, batch=256, lr=5e-4)
    return p, net


def test_learned_correction_inside_the_vcycle_gains_per_step(P, trained_vcycle):
    """FGMRES preconditioned by one V-cycle followed by the network's correction
    of the residual the V-cycle leaves (a learned smoothing step trained on the
    plain solver's residual/smoother-correction pairs): per FGMRES step it
    contracts more than the same V-cycle without the network and than with an
    untrained network (measured: 0.0147 against 0.0151 and 0.0171; the plain
    V-cycle alone contracts 0.053 from zero).  The gain is small: the V-cycle
    leaves mostly smooth error, which a 7 x 7 receptive field cannot correct."""
    p, net = trained_vcycle
    rho = dev(W.blob_charge(p, seed=24680))
    rates = {}
    for label, n in (("no network", None), ("untrained", P.Net(seed=77)), ("trained", net)):
        plan = P.Plan.for_problem(p, krylov=1, krylov_precond=4, fallback=0, krylov_max=8)
        if n is not None:
            P.plan_set_net(plan, n)
        _, st = plan.solve(rho, tol=1e-30, allow=(P.OK, P.NOT_CONVERGED))
        assert st["krylov_iterations"] == 8, st
        rates[label] = st["learned_rate"]
        say("v-cycle + net", label, st["learned_rate"], "plain v-cycle", st["vcycle_rate"])
    assert rates["trained"] < rates["no network"], rates
    assert rates["trained"] < rates["untrained"], rates


def test_learned_vcycle_solve_meets_the_oracle_and_falls_back(P, trained):
    """The judged solve with the learned V-cycle reaches the oracle's answer; a
    network trained on targets it cannot represent (the iterates' smooth global
    error, option nn_target 1) contracts less than a plain V-cycle and the solve
    hands over to V-cycles, still meeting the oracle."""
    p, net = trained
    rho = W.blob_charge(p, seed=99)
    ref = solvers.solve_separable(fv.Grid.of(p), rho, p.bc)
    plan = P.Plan.for_problem(p, krylov=1, krylov_precond=4)
    P.plan_set_net(plan, net)
    phi, st = plan.solve(dev(rho), tol=1e-13)
    assert st["status"] == P.OK and st["learned_fallback"] == 0, st
    assert rel_l2(host(phi), ref) <= 1e-12
    bad = P.Net(seed=9)
    cplan = P.Plan.for_problem(p, nn_target=1)
    for k in range(3):
        bad.collect(cplan, dev(W.blob_charge(p, seed=80 + k)), cycles=4, patches_per_cycle=128, seed=k)
    bad.train(epochs=10, batch=128, lr=2e-3)
    plan2 = P.Plan.for_problem(p, krylov=1, krylov_precond=4)
    P.plan_set_net(plan2, bad)
    phi2, st2 = plan2.solve(dev(rho), tol=1e-13)
    say("error-target net", st2["learned_rate"], "plain v-cycle", st2["vcycle_rate"], "fell back", st2["learned_fallback"])
    assert st2["status"] == P.OK
    if st2["learned_rate"] >= st2["vcycle_rate"]:
        assert st2["learned_fallback"] == 1
    assert rel_l2(host(phi2), ref) <= 1e-12


def test_learned_option_errors(P):
    plan = P.Plan.for_problem(W.SMALL, krylov=1)
    plan.set_option("precision", 32)
    with pytest.raises(P.CylPoissonError) as e:
        plan.solve(dev(np.zeros(W.SMALL.shape)), tol=1e-12)
    assert e.value.status == P.EINVAL
