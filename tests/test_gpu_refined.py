"""QMC_REFINED, the mixed path held to the oracle: int8-refined geminal
products (evaluation and the P rebuilds between moves) and screened FP64
proposals.

* Evaluation: log|Psi|, E_kin, E_loc within 1e-8 (the mixed bar of these tests;
  the mixed path's bar is 1e-6) and drift within 1e-8 of the oracle.
* Proposals: ratios of host-driven proposals against the oracle's full
  re-evaluations (1e-8), with and without the drift at r' (the drift request
  takes the dense FP64 rows); the screening really skips functions and keeps
  some.
* Chains: Metropolis chains (device accept) equal the oracle's chain on the
  same draws: positions bitwise, the tracked log|Psi| within 1e-8.
* Refusals: a Pfaffian member of a multi-system group (polarized systems, the
  Pfaffian and multi-system groups are built: their own test files).
"""
import dataclasses

import numpy as np
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu


def _walkers(P, w, Wk):
    sysh = P.JAGPSystem(w.system, precision=P.QMC_REFINED)
    return sysh, P.Walkers(sysh, Wk, adjoint=False)


@pytest.mark.parametrize("name", ["tiny", "mol160"])
def test_refined_eval_matches_oracle(name):
    P = need_gpu()
    if name == "tiny":
        w, Wk = C.tiny_3nuc_10e(), 64
    else:
        w, Wk = C.mol_40nuc_160e(n_walkers=8), 8
    _, wk = _walkers(P, w, Wk)
    r = torch.tensor(w.r0[:Wk])
    out = wk.eval_batch(r.cuda())
    torch.cuda.synchronize()
    ref = O.evaluate(O.from_workload_system(w.system), r)
    e = {k: rel_err(out[k].cpu(), ref[k]).max().item() for k in ("logabs", "e_kin", "e_loc")}
    e_dr = ((out["drift"].cpu() - ref["drift"]).abs() / ref["drift"].abs().clamp(min=1.0)).max().item()
    print(f"[refined eval {name}] {e} drift {e_dr:.3e}")
    assert max(e.values()) <= 1e-8 and e_dr <= 1e-8
    assert torch.equal(out["sign"].cpu(), ref["sign"])


@pytest.mark.parametrize("drift", [False, True])
def test_refined_host_proposals_match_oracle(drift):
    P = need_gpu()
    w = C.mol_40nuc_160e(n_walkers=8)
    _, wk = _walkers(P, w, 8)
    r = torch.tensor(w.r0)
    sy = O.from_workload_system(w.system)
    disp = torch.tensor(C.chain_arrays(31, 4, 8)[0])
    kept = []
    for t, e in enumerate((5, 79, 80, 150)):
        wk.eval_batch(r.cuda())
        rn = r[:, e] + disp[t]
        res = wk.propose(e, rn.cuda().contiguous(), drift=drift)
        ratio = res[0] if drift else res
        torch.cuda.synchronize()
        rr = O.move_ratio(sy, r, e, rn)
        err = rel_err(ratio.cpu(), rr).max().item()
        print(f"[refined propose e={e} drift={drift}] max rel err {err:.3e}")
        assert err <= 1e-8
        if drift:
            r2 = r.clone()
            r2[:, e] = rn
            d_ref = O.evaluate(sy, r2)["drift"][:, e]
            assert ((res[1].cpu() - d_ref).abs() / d_ref.abs().clamp(min=1.0)).max().item() <= 1e-6
        else:
            kept.append(wk.read(P.STATE_KEPT).cpu())
    if kept:
        k = torch.stack(kept)
        frac = (k / w.system.lam.shape[0]).mean().item()
        print(f"[refined screening] basis functions streamed per proposal: {k.mean().item():.1f} "
              f"of {w.system.lam.shape[0]} ({100 * frac:.1f} %)")
        assert 0.0 < frac < 1.0


@pytest.mark.parametrize("name", ["tiny", "mol160"])
def test_refined_chain_matches_oracle(name):
    P = need_gpu()
    if name == "tiny":
        w, Wk, n_steps = C.tiny_3nuc_10e(n_walkers=16, n_steps=200), 16, 200
        d, u = w.disp, w.unif
    else:
        w, Wk, n_steps = C.mol_40nuc_160e(n_walkers=4), 4, 48
        d, u = C.chain_arrays(77, n_steps, Wk)
    _, wk = _walkers(P, w, Wk)
    r0 = torch.tensor(w.r0[:Wk])
    wk.eval_batch(r0.cuda())
    acc = torch.zeros(Wk, dtype=torch.int32, device="cuda")
    wk.vmc_steps(0, torch.tensor(d, device="cuda"), torch.tensor(u, device="cuda"), acc)
    rg = wk.read(P.STATE_R).cpu()
    la = wk.read(P.STATE_LOGABS).cpu()
    torch.cuda.synchronize()
    sy = O.from_workload_system(w.system)
    rf, _, accs = O.run_chain(sy, r0, torch.tensor(d), torch.tensor(u))
    print(f"[refined chain {name}] accepted {int(acc.sum())} of {Wk * n_steps} (oracle {int(accs.sum())})")
    assert torch.equal(rg, rf)
    assert int(acc.sum()) == int(accs.sum())
    assert rel_err(la, O.log_psi(sy, rf)[0]).max().item() <= 1e-8


def test_refined_refusals():
    # a QMC_REFINED Pfaffian is built, but not as a member of a multi-system group
    P = need_gpu()
    w = C.pfaffian_4nuc_20e(n_walkers=4)
    sysh = P.JAGPSystem(w.system, precision=P.QMC_REFINED)
    wk = P.Walkers(sysh, 4, adjoint=False)
    wk.eval_batch(torch.tensor(w.r0[:4], device="cuda"))
    with pytest.raises(P.QMCError) as ei:
        P.MultiSystem([wk])
    assert ei.value.code == -5


def test_refined_far_proposal_keeps_nothing_and_ratio_is_zero():
    # A proposal 1000 bohr from every nucleus: every basis value at r' is 0 in
    # FP64 (e^{-zeta r^2} underflows), so the screening keeps no function and
    # the determinant ratio is exactly 0, as the oracle's (the Jastrow factor
    # stays finite); the device Metropolis rejects it.
    P = need_gpu()
    w = C.mol_40nuc_160e(n_walkers=4)
    _, wk = _walkers(P, w, 4)
    r = torch.tensor(w.r0)
    wk.eval_batch(r.cuda())
    rn = r[:, 11].clone()
    rn[:, 0] += 1000.0
    ratio = wk.propose(11, rn.cuda().contiguous())
    kept = wk.read(P.STATE_KEPT).cpu()
    torch.cuda.synchronize()
    ref = O.move_ratio(O.from_workload_system(w.system), r, 11, rn)
    print(f"[refined far proposal] kept {kept.tolist()} ratio {ratio.cpu().tolist()} oracle {ref.tolist()}")
    assert (kept == 0).all()
    assert (ratio.cpu() == 0.0).all() and (ref == 0.0).all()


@pytest.mark.parametrize("Wk", [1, 13])
def test_refined_ragged_walker_counts(Wk):
    # one walker, and 13 walkers (1040 rows of the int8 products: a partial
    # 128-row tile; walker count not a multiple of the 8 XCDs): evaluation and
    # a 40-step chain against the oracle
    P = need_gpu()
    w = C.mol_40nuc_160e(n_walkers=Wk)
    _, wk = _walkers(P, w, Wk)
    r = torch.tensor(w.r0[:Wk])
    out = wk.eval_batch(r.cuda())
    d, u = C.chain_arrays(91, 40, Wk)
    wk.vmc_steps(70, torch.tensor(d, device="cuda"), torch.tensor(u, device="cuda"))
    rg = wk.read(P.STATE_R).cpu()
    torch.cuda.synchronize()
    sy = O.from_workload_system(w.system)
    ref = O.evaluate(sy, r)
    assert rel_err(out["e_loc"].cpu(), ref["e_loc"]).max().item() <= 1e-8
    rf, _, _ = O.run_chain(sy, r, torch.tensor(d), torch.tensor(u), e_start=70)
    assert torch.equal(rg, rf)
