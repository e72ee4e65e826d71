"""QMC_REFINED with unpaired orbitals (polarized AGP, eq:wfAGPunpaired): the
int8-refined P products, and screened proposals whose up moves stream the
down electrons' rows followed by the unpaired orbitals' values (both kept
transposed per walker, the column maxima of the screening taken over both).

Cases: polarized_4nuc_20e (11 up / 9 down, two unpaired orbitals; an odd row
count: the plain screened kernel) and the same system with 12 up / 10 down
(an even row count: the blocked screened stream and the persistent sweep).

* Evaluation within 1e-8 of the oracle (log|Psi|, E_kin, E_loc, drift).
* Host-driven proposals of up and down electrons: ratios within 1e-8 of the
  oracle's full re-evaluations, with and without the drift at r'; the
  screening keeps some functions and skips some.
* Chains equal the oracle's chains (positions bitwise, accept counts), the
  tracked log|Psi| within 1e-8; a fresh evaluation afterwards within 1e-8.
"""
import dataclasses

import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu


def _case(name, Wk):
    w = C.polarized_4nuc_20e(n_walkers=max(Wk, 32))
    if name == "odd":
        return w.system, torch.tensor(w.r0[:Wk]), w
    s = dataclasses.replace(w.system, n_up=12, n_dn=10)
    return s, torch.tensor(C.random_positions(53, s, Wk)), w


def _walkers(P, s, Wk):
    sysh = P.JAGPSystem(s, precision=P.QMC_REFINED)
    return sysh, P.Walkers(sysh, Wk, adjoint=False)


@pytest.mark.parametrize("name", ["odd", "even"])
def test_refined_polarized_eval(name):
    P = need_gpu()
    s, r, _ = _case(name, 32)
    _, wk = _walkers(P, s, 32)
    out = wk.eval_batch(r.cuda())
    torch.cuda.synchronize()
    ref = O.evaluate(O.from_workload_system(s), r)
    e = {k: rel_err(out[k].cpu(), ref[k]).max().item() for k in ("logabs", "e_kin", "e_loc")}
    e_dr = ((out["drift"].cpu() - ref["drift"]).abs() / ref["drift"].abs().clamp(min=1.0)).max().item()
    print(f"[refined polarized eval {name}] {e} drift {e_dr:.3e}")
    assert max(e.values()) <= 1e-8 and e_dr <= 1e-8
    assert torch.equal(out["sign"].cpu(), ref["sign"])


@pytest.mark.parametrize("drift", [False, True])
@pytest.mark.parametrize("name", ["odd", "even"])
def test_refined_polarized_proposals(name, drift):
    P = need_gpu()
    Wk = 16
    s, r, _ = _case(name, Wk)
    _, wk = _walkers(P, s, Wk)
    sy = O.from_workload_system(s)
    N = s.n_up + s.n_dn
    disp = torch.tensor(C.chain_arrays(37, 4, Wk)[0])
    kept = []
    for t, e in enumerate((0, s.n_up - 1, s.n_up, N - 1)):
        wk.eval_batch(r.cuda())
        rn = r[:, e] + disp[t]
        res = wk.propose(e, rn.cuda().contiguous(), drift=drift)
        ratio = res[0] if drift else res
        torch.cuda.synchronize()
        err = rel_err(ratio.cpu(), O.move_ratio(sy, r, e, rn)).max().item()
        print(f"[refined polarized {name} e={e} drift={drift}] {err:.3e}")
        assert err <= 1e-8, (e, err)
        if drift:
            r2 = r.clone()
            r2[:, e] = rn
            d_ref = O.evaluate(sy, r2)["drift"][:, e]
            assert ((res[1].cpu() - d_ref).abs() / d_ref.abs().clamp(min=1.0)).max().item() <= 1e-6
        else:
            kept.append(wk.read(P.STATE_KEPT).cpu())
    if kept:
        frac = (torch.stack(kept) / s.lam.shape[0]).mean().item()
        print(f"[refined polarized {name}] share of basis functions streamed {frac:.3f}")
        assert 0.0 < frac <= 1.0


@pytest.mark.parametrize("name", ["odd", "even"])
def test_refined_polarized_chain_matches_oracle(name):
    P = need_gpu()
    Wk, n_steps = 16, 200
    s, r0, w = _case(name, Wk)
    d, u = (w.disp[:n_steps, :Wk], w.unif[:n_steps, :Wk]) if name == "odd" else C.chain_arrays(59, n_steps, Wk)
    _, wk = _walkers(P, s, Wk)
    wk.eval_batch(r0.cuda())
    acc = torch.zeros(Wk, dtype=torch.int32, device="cuda")
    wk.vmc_steps(0, torch.tensor(d, device="cuda").contiguous(), torch.tensor(u, device="cuda").contiguous(), acc)
    rg = wk.read(P.STATE_R).cpu()
    la = wk.read(P.STATE_LOGABS).cpu()
    torch.cuda.synchronize()
    sy = O.from_workload_system(s)
    rf, _, accs = O.run_chain(sy, r0, torch.tensor(d), torch.tensor(u))
    print(f"[refined polarized chain {name}] accepted {int(acc.sum())} of {Wk * n_steps}")
    assert torch.equal(rg, rf)
    assert int(acc.sum()) == int(accs.sum())
    assert rel_err(la, O.log_psi(sy, rf)[0]).max().item() <= 1e-8
    out = wk.eval_batch(rg.cuda())
    torch.cuda.synchronize()
    ref = O.evaluate(sy, rf)
    assert rel_err(out["e_loc"].cpu(), ref["e_loc"]).max().item() <= 1e-8
