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


def test_learned_option_errors(P):
    plan = P.Plan.for_problem(W.SMALL, krylov=1)
    plan.set_option("precision", 32)
    with pytest.raises(P.CylPoissonError) as e:
        plan.solve(dev(np.zeros(W.SMALL.shape)), tol=1e-12)
    assert e.value.status == P.EINVAL
