"""Pfaffian wave function in QMC_REFINED: the evaluation's B rows
(B^s_j = psi(r_j)^T K^{s s_j}) come from the error-free int8 digit products,
everything after them (G~, Pf, G~^{-1}, the cofactor vectors, moves) is the
FP64 Pfaffian path.

* G~ equals the FP64 path's G~ to 1e-13 of its largest entry (the digit
  expansion's truncation is 7e-14 of max|phi| max|K| L per product).
* The evaluation matches the oracle at the refined bars (1e-8 relative on
  log|Psi|, E_kin, E_loc and the drift), signs equal.
* A 100-step chain equals the oracle's chain (positions bitwise, accept counts).
* New pairing coefficients (set_params, set_pfaffian) reach the digits: the
  re-evaluated walkers match the oracle of the changed system.
"""
import dataclasses

import numpy as np
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fw():
    return C.pfaffian_4nuc_20e()


def _balanced(s):
    L_ = len(s.lam)
    return dataclasses.replace(s, n_up=10, n_dn=10, unpaired=np.zeros((L_, 0)), unpaired_dn=np.zeros((L_, 0)))


def _eval(P, s, r0, Wk, precision):
    sysh = P.JAGPSystem(s, precision=precision)
    wk = P.Walkers(sysh, Wk)
    r = torch.tensor(r0[:Wk], device="cuda")
    out = wk.eval_batch(r)
    torch.cuda.synchronize()
    return sysh, wk, r.cpu(), out


def _check(out, ref, label, bar=1e-8):
    e = {k: rel_err(out[k].cpu(), ref[k]).max().item() for k in ("logabs", "e_kin", "e_loc")}
    d = out["drift"].cpu()
    e_dr = ((d - ref["drift"]).abs() / ref["drift"].abs().clamp(min=1.0)).max().item()
    print(f"[refined pfaffian {label}] {e} drift {e_dr:.3e}")
    assert max(e.values()) <= bar and e_dr <= bar
    assert torch.equal(out["sign"].cpu(), ref["sign"])
    assert int(out["status"].abs().max()) == 0


@pytest.mark.parametrize("case", ["unpaired_k2", "balanced"])
def test_refined_pfaffian_eval(fw, case):
    P = need_gpu()
    s = fw.system if case == "unpaired_k2" else _balanced(fw.system)
    r0 = fw.r0 if case == "unpaired_k2" else C.random_positions(43, s, 32)
    _, wr, r, outr = _eval(P, s, r0, 32, P.QMC_REFINED)
    _, wf, _, outf = _eval(P, s, r0, 32, P.QMC_FP64)
    Gr, Gf = wr.read(P.STATE_W).cpu(), wf.read(P.STATE_W).cpu()
    assert torch.equal(Gr, -Gr.transpose(1, 2))
    dG = ((Gr - Gf).abs().max() / Gf.abs().max()).item()
    print(f"[refined pfaffian {case}] G~ against the FP64 path {dG:.3e}")
    assert dG <= 1e-13
    _check(outr, O.evaluate(O.from_workload_system(s), r), case)
    assert rel_err(outr["logabs"].cpu(), outf["logabs"].cpu()).max().item() <= 1e-12


def test_refined_pfaffian_chain_matches_oracle(fw):
    P = need_gpu()
    Wk, T = 16, 100
    _, wk, r, _ = _eval(P, fw.system, fw.r0, Wk, P.QMC_REFINED)
    disp = torch.tensor(fw.disp[:T, :Wk]).contiguous()
    unif = torch.tensor(fw.unif[:T, :Wk]).contiguous()
    cnt = torch.zeros(Wk, dtype=torch.int32, device="cuda")
    wk.vmc_steps(0, disp.cuda(), unif.cuda(), cnt)
    rg = wk.read(P.STATE_R).cpu()
    la = wk.read(P.STATE_LOGABS).cpu()
    torch.cuda.synchronize()
    sy = O.from_workload_system(fw.system)
    rf, _, accs = O.run_chain(sy, r, disp, unif)
    assert torch.equal(rg, rf)
    assert torch.equal(cnt.cpu(), accs.sum(0).to(torch.int32))
    assert rel_err(la, O.evaluate(sy, rf)["logabs"]).max().item() <= 1e-8
    # a later evaluation from scratch at the chain's positions
    out = wk.eval_batch(rg.cuda())
    torch.cuda.synchronize()
    _check(out, O.evaluate(sy, rf), "after a chain")


def test_refined_pfaffian_parameter_updates(fw):
    P = need_gpu()
    sysh, wk, r, _ = _eval(P, fw.system, fw.r0, 8, P.QMC_REFINED)
    s = fw.system
    rng = np.random.default_rng(47)
    L_ = len(s.lam)
    lam2 = s.lam + 0.05 * rng.standard_normal(s.lam.shape)
    a = rng.standard_normal((L_, L_))
    uu2 = s.pf_uu + 0.03 * (a - a.T)
    b = rng.standard_normal((L_, L_))
    dd2 = s.pf_dd + 0.03 * (b - b.T)
    T = lambda x: torch.tensor(np.ascontiguousarray(x), device="cuda")
    sysh.set_params(lam=T(lam2))
    out = wk.eval_batch(r.cuda())
    torch.cuda.synchronize()
    _check(out, O.evaluate(O.from_workload_system(dataclasses.replace(s, lam=lam2)), r), "new A^ud")
    sysh.set_pfaffian(pf_uu=T(uu2), pf_dd=T(dd2))
    out = wk.eval_batch(r.cuda())
    torch.cuda.synchronize()
    s2 = dataclasses.replace(s, lam=lam2, pf_uu=uu2, pf_dd=dd2)
    _check(out, O.evaluate(O.from_workload_system(s2), r), "new same-spin blocks")


def test_refined_pfaffian_80_electrons():
    # pfaffian_20nuc_80e (G~ 80 x 80, L = 300) on sampled walkers
    P = need_gpu()
    w = C.pfaffian_20nuc_80e(n_walkers=64)
    _, wk, r, out = _eval(P, w.system, w.r0, 64, P.QMC_REFINED)
    idx = [0, 21, 42, 63]
    ref = O.evaluate(O.from_workload_system(w.system), r[idx])
    sub = {k: v[idx] for k, v in out.items()}
    _check(sub, ref, "80 electrons")
