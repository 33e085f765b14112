"""GPU: one round of the pipeline -- Alg. 3's output transforms, the non-parametric update
(eq. 2), T iterations from the current state, and the reverse mode back to the raw predictions --
against the FP64 oracle (oracle.param_transform, nonparam_update, unrolled_grad from a state)."""
import numpy as np
import pytest

import synth
from tests.gpu_util import host, make_instance, say
from tests.test_gpu_adjoint import (MIN_DETERMINED, close_bounded, close_grad, euler_close, f32, gpu_states,
                                     trajectory_tolerances)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    oracle.build(force=False)
    return oracle


def dev(a):
    import torch
    return torch.tensor(np.asarray(a, np.float32), device="cuda")


def raw(p, seed):
    rng = np.random.default_rng(seed)
    return (f32(rng.normal(size=p.nnz)), f32(rng.normal(0, 0.3, size=p.nnz)), f32(rng.normal(0, 0.2, size=p.nnz)))


def test_param_transform_and_vjp_match_oracle(orc):
    p = synth.workload("gm", small=True)["problem"]
    inst, _, _ = make_instance(p)
    wh, ah, th = raw(p, 1)
    w, a, t = (host(x) for x in inst.param_transform(dev(wh), dev(ah), dev(th)))
    wo, ao, to = orc.param_transform(p, wh, ah, th)
    np.testing.assert_allclose(w, wo, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(a, ao, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(t, to, rtol=1e-5, atol=1e-6)
    g = [f32(np.random.default_rng(2 + k).normal(size=p.nnz)) for k in range(3)]
    got = [host(x) for x in inst.param_transform_vjp(dev(w), dev(a), *[dev(x) for x in g])]
    ref = orc.param_transform_vjp(p, w, a, *g)
    for x, r in zip(got, ref):
        np.testing.assert_allclose(x, r, rtol=1e-5, atol=1e-6)
    # no theta: the other two outputs only
    w2, a2, t2 = inst.param_transform(dev(wh), dev(ah))
    assert t2 is None
    np.testing.assert_array_equal(host(w2), w)


def test_nonparam_update_matches_oracle_and_keeps_feasibility(orc):
    p = synth.workload("setcover")["problem"]
    om, ah, th = raw(p, 3)
    inst, _, alt = make_instance(p, 1 / (1 + np.exp(-om)), ah)
    inst.run(3)
    lam, M = (host(x) for x in inst.get_state())
    inst.nonparam_update(dev(th))
    lam2, M2 = (host(x) for x in inst.get_state())
    np.testing.assert_array_equal(M2, M)
    np.testing.assert_allclose(lam2, orc.nonparam_update(p, lam, th), rtol=1e-6, atol=1e-6)
    var = p.col.astype(np.int64)
    t1, t2 = np.zeros(p.n), np.zeros(p.n)
    np.add.at(t1, var, lam + M)
    np.add.at(t2, var, lam2 + M2)
    np.testing.assert_allclose(t2, t1, atol=1e-5)
    # the bound afterwards is the oracle's at the updated state
    lb = inst.lower_bound()[0]
    assert lb == pytest.approx(orc.lower_bound(p, host(alt), lam2, M2)[0], rel=1e-5)


@pytest.mark.parametrize("case,T,K,seed", [("mixed", 3, 2, 10), ("setcover", 4, 3, 11), ("gm-small", 3, 1, 7)])
def test_unrolled_from_state_matches_oracle(orc, case, T, K, seed):
    p = {"mixed": lambda: synth.random_tiny(0, n=40, m=60, kmin=1, kmax=14, amin=-7, amax=7),
         "setcover": lambda: synth.workload("setcover")["problem"],
         "gm-small": lambda: synth.workload("gm", small=True)["problem"]}[case]()
    wh, ah, th = raw(p, seed)
    om = f32(1 / (1 + np.exp(-wh)))
    inst, _, alt = make_instance(p, om, ah)
    al = host(alt)
    inst.run(2)
    inst.nonparam_update(dev(th))
    start = tuple(t.clone() for t in inst.get_state())
    lam0, M0 = (host(x) for x in start)
    pc = synth.Problem(p.n, f32(p.c), p.row_ptr, p.col, p.coef, p.sense, p.rhs)
    states_g = gpu_states(inst, T, start=start)
    states_o = orc.trajectory(pc, om, al, T, lam0=lam0, M0=M0)
    ptol = trajectory_tolerances(pc, al, states_g, states_o, orc)
    lb = inst.forward_unrolled_from_state(T, K)
    dw, da, dl0, dm0 = (host(x) for x in inst.backward_state(1.0))
    lb_o, dw_o, da_o, (dl0_o, dm0_o), (bw, ba, (bl0, bm0), ws) = orc.unrolled_grad(pc, om, al, T, lam0=lam0, M0=M0,
                                                                                   pass_tol=ptol)
    assert lb == pytest.approx(lb_o, rel=1e-5, abs=1e-6)
    unc = np.bincount(p.col, minlength=p.n) == 0
    terms = np.concatenate([dl0 * lam0, dm0 * M0])
    euler_close(terms.sum(), lb - np.minimum(pc.c[unc], 0).sum(), np.abs(terms).sum(), "Euler from a state")
    det = [close_bounded(g, ref, b, nm, sc) for g, ref, b, nm, sc in
           zip((dw, da, dl0, dm0), (dw_o, da_o, dl0_o, dm0_o), (bw, ba, bl0, bm0),
               ("d_omega", "d_alpha", "d_lam0", "d_M0"), (ws, None, None, None))]
    say(f"  {case}: determined entries " + " ".join(f"{d:.3f}" for d in det))
    assert min(det) >= MIN_DETERMINED
    # the instance is at the end of the round: the bound is unchanged
    assert inst.lower_bound()[0] == pytest.approx(lb, rel=1e-6)


def test_dual_round_autograd(orc):
    import torch

    from paper_2205_11638_amd.autograd import dual_round
    p = synth.workload("gm", small=True)["problem"]
    inst, _, _ = make_instance(p)
    wh, ah, th = raw(p, 9)
    # an earlier round (no gradients)
    inst.set_params(*inst.param_transform(dev(wh), dev(ah))[:2])
    inst.run(2)
    lam_prev, M_prev = (host(x) for x in inst.get_state())
    W, A, Th = (torch.tensor(np.asarray(x, np.float32), device="cuda", requires_grad=True) for x in (wh, ah, th))
    lb = dual_round(inst, W, A, Th, 3, 2)
    (-lb).backward()
    om, al, _ = orc.param_transform(p, wh, ah, th)
    al32 = f32(al)
    lam0 = orc.nonparam_update(p, lam_prev, th)
    # the GPU's trajectory of the round: its start state is the updated one, re-formed from the
    # state before the update (the round left the instance at its end)
    inst.set_state(dev(lam_prev), dev(M_prev))
    inst.nonparam_update(dev(th))
    start = tuple(t.clone() for t in inst.get_state())
    states_g = gpu_states(inst, 3, start=start)
    states_o = orc.trajectory(p, f32(om), al32, 3, lam0=lam0, M0=M_prev)
    ptol = trajectory_tolerances(p, al32, states_g, states_o, orc)
    lb_o, dw_o, da_o, (dl0_o, _), bnd = orc.unrolled_grad(p, f32(om), al32, 3, lam0=lam0, M0=M_prev, pass_tol=ptol)
    assert lb.item() == pytest.approx(lb_o, rel=1e-5)
    assert not (bnd[0].any() or bnd[1].any() or bnd[2][0].any())  # every decision of this round is unique
    dwh, dah, dth = orc.param_transform_vjp(p, f32(om), al32, dw_o, da_o, dl0_o)
    close_grad(-host(W.grad), dwh, "d_omega_hat")
    close_grad(-host(A.grad), dah, "d_alpha_hat")
    close_grad(-host(Th.grad), dth, "d_theta_hat")


def test_dual_round_stored_trajectory_matches_checkpoints():
    """A round with the whole trajectory kept (ckpt_every = -1) gives the bound and the gradients of the
    three raw predictions of checkpoints every iteration, bit for bit."""
    import torch

    from paper_2205_11638_amd.autograd import dual_round
    p = synth.workload("gm", small=True)["problem"]
    inst, _, _ = make_instance(p)
    wh, ah, th = raw(p, 11)
    inst.set_params(*inst.param_transform(dev(wh), dev(ah))[:2])
    inst.run(2)
    lam, M = inst.get_state()
    lam, M = lam.clone(), M.clone()
    out = []
    for K in (1, -1):
        inst.set_state(lam, M)
        W, A, Th = (torch.tensor(np.asarray(x, np.float32), device="cuda", requires_grad=True) for x in (wh, ah, th))
        lb = dual_round(inst, W, A, Th, 4, K)
        (-lb).backward()
        out.append((lb.item(), host(W.grad), host(A.grad), host(Th.grad)))
    assert out[0][0] == out[1][0]
    for a, b in zip(out[0][1:], out[1][1:]):
        np.testing.assert_array_equal(a, b)


def test_d_c_needs_a_reset_start():
    import paper_2205_11638_amd as dd
    p = synth.workload("setcover")["problem"]
    inst, _, _ = make_instance(p)
    inst.forward_unrolled_from_state(2)
    with pytest.raises(dd.DDError) as e:
        inst.backward(1.0)
    assert e.value.code == dd.binding.DD_E_ARG
    inst.backward_state(1.0)  # the record is still valid
