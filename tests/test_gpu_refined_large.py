"""The refined mixed path (QMC_REFINED) on the 1024-electron workload: 256
nuclei, L = 4096, Lambda banded at 8 bohr (the int8 digit products skip
Lambda's zero tiles as the FP64 product does), n = 512 per spin (blocked
inverse, refresh after 64 moves of one spin, the unstaged set-up and the
wide screened proposal kernel).

* Evaluation against the oracle at the mixed bar used by every refined test
  (1e-8 relative on log|Psi| and E_loc; the mixed path's bar is 1e-6).
* Proposal ratios of up and down electrons against the oracle's ratio of two
  full evaluations (1e-8), with the screened kept count strictly inside (0, L).
* 24 Metropolis steps of two walkers: positions equal to the oracle's chain on
  the same draws (accept decisions identical), and the tracked log|Psi| equal to
  a fresh FP64 evaluation at the final positions (1e-8).
"""
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu

WK = 2


@pytest.fixture(scope="module")
def large():
    P = need_gpu()
    w = C.large_256nuc_1024e(n_walkers=WK)
    sysh = P.JAGPSystem(w.system, precision=P.QMC_REFINED)
    wk = P.Walkers(sysh, WK, adjoint=False)
    yield P, w, sysh, wk
    wk.close()
    sysh.close()


def test_refined_large_eval_matches_oracle(large):
    P, w, sysh, wk = large
    r = torch.tensor(w.r0[:WK])
    out = wk.eval_batch(r.cuda(), drift=True)
    torch.cuda.synchronize()
    ref = O.evaluate(O.from_workload_system(w.system), r)
    e_la = rel_err(out["logabs"].cpu(), ref["logabs"]).max().item()
    e_el = rel_err(out["e_loc"].cpu(), ref["e_loc"]).max().item()
    print(f"[refined 1024e eval] logabs {e_la:.3e} e_loc {e_el:.3e}")
    assert e_la <= 1e-8 and e_el <= 1e-8
    assert torch.equal(out["sign"].cpu(), ref["sign"])


def test_refined_large_proposals_match_oracle(large):
    P, w, sysh, wk = large
    r = torch.tensor(w.r0[:WK])
    sy = O.from_workload_system(w.system)
    g = torch.Generator().manual_seed(9)
    L = w.system.lam.shape[0]
    for e in (7, 400, 512, 1000):
        wk.eval_batch(r.cuda())
        rn = r[:, e] + 0.3 * torch.randn(WK, 3, generator=g, dtype=torch.float64)
        ratio = wk.propose(e, rn.cuda().contiguous())
        kept = wk.read(P.STATE_KEPT).cpu()
        torch.cuda.synchronize()
        ref = O.move_ratio(sy, r, e, rn)
        err = rel_err(ratio.cpu(), ref).max().item()
        print(f"[refined 1024e propose e={e}] ratio err {err:.3e}, kept {kept.tolist()} of {L}")
        assert err <= 1e-8
        assert (kept > 0).all() and (kept < L).all()


def test_refined_large_chain_matches_oracle(large):
    P, w, sysh, wk = large
    n_steps = 24
    d, u = C.chain_arrays(505, n_steps, WK)
    r0 = torch.tensor(w.r0[:WK])
    wk.eval_batch(r0.cuda())
    acc = torch.zeros(WK, dtype=torch.int32, device="cuda")
    wk.vmc_steps(500, torch.tensor(d, device="cuda"), torch.tensor(u, device="cuda"), acc)
    r_gpu = wk.read(P.STATE_R).cpu()
    la = wk.read(P.STATE_LOGABS).cpu()
    torch.cuda.synchronize()
    sy = O.from_workload_system(w.system)
    r_ref, _, accs = O.run_chain(sy, r0, torch.tensor(d), torch.tensor(u), e_start=500)
    print(f"[refined 1024e chain] accepts gpu {acc.tolist()} oracle {accs.sum(0).tolist()}")
    assert torch.equal(r_gpu, r_ref)
    assert acc.cpu().tolist() == accs.sum(0).tolist()
    fresh = O.evaluate(sy, r_ref)["logabs"]
    assert rel_err(la, fresh).max().item() <= 1e-8
