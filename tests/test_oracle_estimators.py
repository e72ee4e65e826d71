"""Pins of the estimator oracle (Atomic forces and Stochastic reconfiguration
sections): space-warp weights, total derivatives, the reweighting factor and
the SR step, against identities, closed forms and finite differences.
"""
import numpy as np
import torch

from oracle import estimators as E
from oracle import jagp as O
from workloads import configs as C

DT = torch.float64


def _tiny(n=3):
    w = C.tiny_3nuc_10e(n_walkers=n, n_steps=1)
    return w, O.from_workload_system(w.system), torch.tensor(w.r0)


def test_warp_weights_partition_of_unity_and_gradient():
    w, sy, r = _tiny()
    om, gom = E.warp_weights(sy, r)
    assert torch.allclose(om.sum(-1), torch.ones_like(om[..., 0]), rtol=0, atol=1e-14)
    assert torch.allclose(gom.sum(2), torch.zeros_like(gom[:, :, 0]), rtol=0, atol=1e-12)
    h = 1e-6
    for ax in range(3):
        e = torch.zeros(3, dtype=DT); e[ax] = h
        fd = (E.warp_weights(sy, r + e)[0] - E.warp_weights(sy, r - e)[0]) / (2 * h)
        assert torch.allclose(gom[..., ax], fd, rtol=1e-6, atol=1e-8)
    # at a nucleus the weight of that nucleus tends to one
    near = sy.R[1].view(1, 1, 3) + 1e-4
    assert abs(E.warp_weights(sy, near)[0][0, 0, 1].item() - 1.0) < 1e-10


def test_swct_total_derivative_is_derivative_along_the_warp():
    # d/dt e_L(R_a + t u, r_i + t u omega_a(r_i)) at t = 0, central differences
    w, sy, r = _tiny(2)
    pw = O.forces_per_walker(sy, r)
    for which, key in ((0, "logabs"), (1, "e_loc")):
        tot = E.swct_total(sy, r, pw["R"][which], pw["r"][which], jacobian=False)
        for a, ax in ((0, 0), (2, 1)):
            h = 1e-5
            vals = []
            for s in (1.0, -1.0):
                R = sy.R.clone(); R[a, ax] += s * h
                om = E.warp_weights(sy, r)[0][..., a]               # [Wk, N]
                rr = r.clone(); rr[..., ax] += s * h * om
                vals.append(O.evaluate(sy, rr, R=R)[key])
            fd = (vals[0] - vals[1]) / (2 * h)
            assert torch.allclose(tot[:, a, ax], fd, rtol=1e-6, atol=1e-6), (key, a, ax)


def test_swct_translation_sum_rule_and_jacobian_term():
    w, sy, r = _tiny(2)
    pw = O.forces_per_walker(sy, r)
    for which in (0, 1):
        tot = E.swct_total(sy, r, pw["R"][which], pw["r"][which], jacobian=True)
        s = tot.sum(1)
        assert torch.allclose(s, torch.zeros_like(s), rtol=0, atol=1e-8)
    # Jacobian term: d/dt 1/2 log det of the warp map of one electron
    x = r[0, 0].clone()
    a, ax, h = 1, 2, 1e-5
    def warp(pt, t):
        om = E.warp_weights(sy, pt.view(1, 1, 3))[0][0, 0, a]
        q = pt.clone(); q[ax] = q[ax] + t * om
        return q
    def logdet(t):
        J = torch.autograd.functional.jacobian(lambda p: warp(p, t), x)
        return 0.5 * torch.logdet(J)
    fd = (logdet(h) - logdet(-h)) / (2 * h)
    gom = E.warp_weights(sy, x.view(1, 1, 3))[1][0, 0, a, ax]
    assert abs(fd.item() - 0.5 * gom.item()) < 1e-7


def test_reweighting_scale_invariance_and_node_exponent():
    w, sy, r = _tiny(4)
    theta = 3.0 / 8.0
    R1, _ = E.reweight(sy, r, theta, 0.0)
    sy2 = O.from_workload_system(w.system)
    sy2.lam = sy2.lam * 7.5
    R2, _ = E.reweight(sy2, r, theta, 0.0)
    assert torch.allclose(R1, R2, rtol=1e-12)
    # two same-spin electrons approaching each other: W nearly singular,
    # R vanishes as delta^(2 theta)
    vals = []
    for d in (1e-4, 5e-5):
        rr = r[:1].clone()
        rr[0, 1] = rr[0, 0] + d * torch.tensor([0.3, -0.5, 0.8], dtype=DT)
        vals.append(E.reweight(sy, rr, theta, 0.0)[0].item())
    assert abs(vals[1] / vals[0] - 2 ** (-2 * theta)) < 1e-3
    # the regularised weight
    eps = float(R1.median())
    R, wgt = E.reweight(sy, r, theta, eps)
    assert torch.allclose(wgt, torch.where(R >= eps, torch.ones_like(R), (R / eps) ** 2), rtol=1e-14)


def test_sr_step_definitions():
    rng = np.random.default_rng(5)
    M, P = 64, 6
    # centered columns orthogonal: S diagonal, delta_k = f_k / (s_kk (1 + eps))
    X = rng.normal(size=(M, P))
    Q, _ = np.linalg.qr(X - X.mean(0))          # centered, orthonormal columns
    Ok = torch.tensor(Q * np.arange(1, P + 1) + rng.normal(size=P))
    el = torch.tensor(rng.normal(size=M))
    delta, f, S = E.sr_step(Ok, el, 0.1)
    assert torch.allclose(S, S.T)
    assert torch.allclose(S, torch.diag(torch.tensor(np.arange(1, P + 1) ** 2 / M, dtype=DT)), atol=1e-14)
    assert torch.allclose(delta, f / (torch.diagonal(S) * 1.1), rtol=1e-10)
    # a general sample: S positive semi-definite, the step solves S' delta = f
    Og = torch.tensor(rng.normal(size=(M, P)))
    dg, fg, Sg = E.sr_step(Og, el, 0.1)
    assert (torch.linalg.eigvalsh(Sg) > -1e-12).all()
    assert torch.allclose((Sg + 0.1 * torch.diag(torch.diagonal(Sg))) @ dg, fg, rtol=1e-10, atol=1e-12)
    # zero variance: a constant local energy gives no force and no step
    d0, f0, _ = E.sr_step(Ok, torch.full((M,), -3.2, dtype=DT), 0.1)
    assert f0.abs().max() < 1e-12 and d0.abs().max() < 1e-10
    # uniform weights equal no weights; integer weights equal repeated samples
    d1 = E.sr_step(Ok, el, 0.1, torch.full((M,), 2.5, dtype=DT))[0]
    assert torch.allclose(d1, delta, rtol=1e-12)
    wts = torch.tensor(rng.integers(1, 4, size=M), dtype=DT)
    rep = torch.repeat_interleave(torch.arange(M), wts.long())
    d2 = E.sr_step(Ok, el, 0.1, wts)[0]
    d3 = E.sr_step(Ok[rep], el[rep], 0.1)[0]
    assert torch.allclose(d2, d3, rtol=1e-10)
