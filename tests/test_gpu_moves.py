"""Parity of single-electron moves (propose / accept / device Metropolis) with
the CPU oracle, whose ratio is Psi(x')/Psi(x) from two full evaluations.

Tolerances: ratio relative 1e-10 (metric |x-y|/max(|y|,1)); after updates
W^{-1} must match a fresh inverse to 1e-9 of its largest entry; a chain's
final log|Psi| must match a fresh oracle evaluation to 1e-10 relative, and its
positions must be bitwise equal (same accept decisions, same FP64 additions).
"""
import numpy as np
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu


def _setup(P, w, n_walkers=None, refresh_every=None):
    Wk = w.r0.shape[0] if n_walkers is None else n_walkers
    sysh = P.JAGPSystem(w.system, refresh_every=refresh_every)
    wk = P.Walkers(sysh, Wk)
    r = torch.tensor(w.r0[:Wk], device="cuda")
    wk.eval_batch(r)
    return sysh, wk, O.from_workload_system(w.system), torch.tensor(w.r0[:Wk])


@pytest.mark.parametrize("e", [0, 3, 4, 5, 9])
def test_propose_ratio_and_drift_tiny(e):
    P = need_gpu()
    w = C.tiny_3nuc_10e()
    _, wk, sy, r = _setup(P, w)
    rn = r[:, e] + torch.tensor(w.disp[0])
    ratio, dn = wk.propose(e, rn.cuda().contiguous(), drift=True)
    torch.cuda.synchronize()
    ref = O.move_ratio(sy, r, e, rn)
    assert rel_err(ratio.cpu(), ref).max().item() <= 1e-10
    r2 = r.clone(); r2[:, e] = rn
    dref = O.evaluate(sy, r2)["drift"][:, e]
    derr = ((dn.cpu() - dref).abs() / torch.clamp(dref.abs(), min=1.0)).max().item()
    assert derr <= 1e-8


@pytest.mark.parametrize("e,Wk", [(7, 16), (95, 16), (7, 13), (95, 13)])
def test_propose_accept_molecule_160e(e, Wk):
    # Wk = 13: a walker count that is not a multiple of the 8 XCDs (the
    # proposal grid's plain block order)
    P = need_gpu()
    w = C.mol_40nuc_160e(n_walkers=Wk)
    _, wk, sy, r = _setup(P, w)
    disp = torch.tensor(C.chain_arrays(11, 1, Wk)[0][0])
    rn = r[:, e] + disp
    ratio = wk.propose(e, rn.cuda().contiguous())
    acc = torch.tensor([(k + 1) % 2 for k in range(Wk)], dtype=torch.uint8)
    wk.accept(e, acc.cuda())
    A = wk.read(P.STATE_AINV).cpu()
    la = wk.read(P.STATE_LOGABS).cpu()
    torch.cuda.synchronize()
    ref = O.move_ratio(sy, r, e, rn)
    assert rel_err(ratio.cpu(), ref).max().item() <= 1e-10
    r2 = r.clone()
    r2[acc.bool(), e] = rn[acc.bool()]
    o2 = O.evaluate(sy, r2, with_intermediates=True)
    scale = o2["A"].abs().amax(dim=(1, 2), keepdim=True)
    assert ((A - o2["A"]).abs() / scale).max().item() <= 1e-9
    assert rel_err(la, o2["logabs"]).max().item() <= 1e-10


def test_chain_tiny_1000_moves_matches_oracle():
    P = need_gpu()
    w = C.tiny_3nuc_10e()
    _, wk, sy, r = _setup(P, w)
    disp = torch.tensor(w.disp)
    unif = torch.tensor(w.unif)
    cnt = torch.zeros(64, dtype=torch.int32, device="cuda")
    wk.vmc_steps(0, disp.cuda(), unif.cuda(), cnt)
    rg = wk.read(P.STATE_R).cpu()
    la = wk.read(P.STATE_LOGABS).cpu()
    sg = wk.read(P.STATE_SIGN).cpu()
    torch.cuda.synchronize()
    rf, ratios, accs = O.run_chain(sy, r, disp, unif)
    assert torch.equal(cnt.cpu(), accs.sum(0).to(torch.int32))
    assert torch.equal(rg, rf)
    ref = O.evaluate(sy, rf)
    assert rel_err(la, ref["logabs"]).max().item() <= 1e-10
    assert torch.equal(sg, ref["sign"])
    # an eval at the end of the chain reproduces the oracle too
    out = wk.eval_batch(rg.cuda())
    torch.cuda.synchronize()
    assert rel_err(out["e_loc"].cpu(), ref["e_loc"]).max().item() <= 1e-10


def test_chain_refresh_schedules():
    # The refresh re-derives W^{-1} and log|det W| from W by Gauss-Jordan; it
    # never changes accept decisions here.  With refreshes every 1 or 32 moves
    # the tracked log|Psi| meets the 1e-10 bar; with refresh_every = 1000 only
    # the changes of spin refresh (every 5 moves here) and the accumulated
    # log|R| is held to a looser bound.
    P = need_gpu()
    w = C.tiny_3nuc_10e(n_walkers=16, n_steps=200)
    disp = torch.tensor(w.disp)
    unif = torch.tensor(w.unif)
    sy = O.from_workload_system(w.system)
    rf, _, _ = O.run_chain(sy, torch.tensor(w.r0), disp, unif)
    ref = O.log_psi(sy, rf)[0]
    for every, tol in ((1, 1e-10), (32, 1e-10), (1000, 1e-7)):
        _, wk, _, _ = _setup(P, w, refresh_every=every)
        wk.vmc_steps(0, disp.cuda(), unif.cuda())
        rr = wk.read(P.STATE_R).cpu()
        la = wk.read(P.STATE_LOGABS).cpu()
        torch.cuda.synchronize()
        assert torch.equal(rr, rf), every
        assert rel_err(la, ref).max().item() <= tol, (every, rel_err(la, ref).max().item())


def test_chain_molecule_160e_one_sweep():
    P = need_gpu()
    w = C.mol_40nuc_160e(n_walkers=8)
    _, wk, sy, r = _setup(P, w)
    disp, unif = C.chain_arrays(12, 160, 8)
    disp, unif = torch.tensor(disp), torch.tensor(unif)
    wk.vmc_steps(0, disp.cuda(), unif.cuda())
    rg = wk.read(P.STATE_R).cpu()
    la = wk.read(P.STATE_LOGABS).cpu()
    torch.cuda.synchronize()
    rf, _, accs = O.run_chain(sy, r, disp, unif)
    assert torch.equal(rg, rf)
    assert rel_err(la, O.evaluate(sy, rf)["logabs"]).max().item() <= 1e-10
    assert accs.float().mean().item() > 0.05


def test_device_sweep_equals_host_driven_moves():
    # qmc_vmc_steps runs most accepts fused with the next proposal's set-up;
    # the host-driven propose / accept calls run every kernel separately.  Same
    # arithmetic in the same order: positions, log|Psi|, W and W^{-1} agree
    # bitwise over 100 steps (refreshes at 32 moves of one spin and at the
    # change of spin, P rebuilds).
    P = need_gpu()
    w = C.mol_40nuc_160e(n_walkers=16)
    _, wk_a, sy, r = _setup(P, w)
    _, wk_b, _, _ = _setup(P, w)
    n = 100
    e0 = 30
    disp, unif = C.chain_arrays(41, n, 16)
    disp, unif = torch.tensor(disp, device="cuda"), torch.tensor(unif, device="cuda")
    cnt = torch.zeros(16, dtype=torch.int32, device="cuda")
    wk_a.vmc_steps(e0, disp, unif, cnt)
    N = w.system.n_up + w.system.n_dn
    for t in range(n):
        e = (e0 + t) % N
        rcur = wk_b.read(P.STATE_R)
        ratio = wk_b.propose(e, (rcur[:, e] + disp[t]).contiguous())
        wk_b.accept(e, (unif[t] < ratio * ratio).to(torch.uint8))
    torch.cuda.synchronize()
    for item in (P.STATE_R, P.STATE_LOGABS, P.STATE_SIGN, P.STATE_W, P.STATE_AINV):
        a, b = wk_a.read(item), wk_b.read(item)
        torch.cuda.synchronize()
        assert torch.equal(a.cpu(), b.cpu()), item
    assert 0 < int(cnt.sum()) < 16 * n


@pytest.mark.parametrize("prec", ["QMC_FP64", "QMC_REFINED"])
def test_vmc_steps_split_into_calls_equals_one_call(prec):
    # Runs of moves with no refresh, change of spin or P rebuild inside go to
    # one persistent launch; a call boundary ends a run with a plain accept
    # and the next call starts with a separate set-up.  A sweep and a half in
    # one call and in calls of 1, 7, 13 and 32 moves: positions, log|Psi| and
    # the accept counts agree bitwise (the same arithmetic in the same order).
    P = need_gpu()
    w = C.mol_40nuc_160e(n_walkers=16)
    N = w.system.n_up + w.system.n_dn
    n = 240
    disp, unif = C.chain_arrays(77, n, 16)
    disp, unif = torch.tensor(disp, device="cuda"), torch.tensor(unif, device="cuda")
    r0 = torch.tensor(w.r0[:16], device="cuda")
    sysh = P.JAGPSystem(w.system, precision=getattr(P, prec))
    out = []
    for sizes in ([n], [1] * 20 + [7] * 10 + [13] * 6 + [32] * 2 + [n - 20 - 70 - 78 - 64]):
        wk = P.Walkers(sysh, 16, adjoint=False)
        wk.eval_batch(r0)
        cnt = torch.zeros(16, dtype=torch.int32, device="cuda")
        t = 0
        for m in sizes:
            wk.vmc_steps(t % N, disp[t:t + m].contiguous(), unif[t:t + m].contiguous(), cnt)
            t += m
        assert t == n
        out.append((wk.read(P.STATE_R).cpu(), wk.read(P.STATE_LOGABS).cpu(), cnt.cpu()))
        torch.cuda.synchronize()
        wk.close()
    (ra, la, ca), (rb, lb, cb) = out
    assert torch.equal(ra, rb)
    assert torch.equal(ca, cb)
    assert torch.equal(la, lb)
    sysh.close()
