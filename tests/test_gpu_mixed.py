"""Reduced-precision paths.

QMC_W_FP32: basis matrix, P = Phi Lambda and the W products in FP32 on MFMA
with FP32 accumulation; LU, inverse, cofactor products, ratios and
inverse updates in FP64.  Checked against a forward-error bound (must
hold).  With u = 2^-24 and gamma = (2L + 4) u (rounding of Phi and Lambda to
FP32, the length-L FP32 accumulation of P and its FP32 storage; the W product
itself accumulates in FP64 and is covered with room to spare), every geminal
entry obeys to first order
    |dW| <= gamma |Phi_up| |Lambda| |Phi_dn|^T
and the derivative rows V = Q_up Lambda Phi_dn^T + Phi_up Lambda Q_dn^T
(Q = lap Phi + 2 grad Phi . grad J, whose trace against W^{-1} is the
determinant part of the kinetic energy) obey the same with |Q| in place of
|Phi|.  Hence, to first order,
    |d log|det W||  <= sum |A^T| * |dW|
    |d e_kin|       <= 1/2 ( sum |(A V A)^T| * |dW| + sum |A^T| * |dV| ).
The bounds are evaluated from the oracle's FP64 quantities.  Condition numbers
of 1e5..1e6 in these workloads amplify u, so this mode alone misses a relative
1e-6 on some walkers.

QMC_MIXED: the same FP32 move path, but each evaluation builds Phi, P, W and the
cofactor products in FP64 and only stores FP32 copies for the moves.  It must
meet relative 1e-6 on log|Psi| and E_loc against the oracle (it reaches FP64
accuracy), and its move ratios obey the FP32 bound above.
"""
import dataclasses

import numpy as np
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu


def _gpu_eval(P, w, precision=None):
    sysh = P.JAGPSystem(w.system, precision=P.QMC_W_FP32 if precision is None else precision)
    wk = P.Walkers(sysh, w.r0.shape[0])
    out = wk.eval_batch(torch.tensor(w.r0, device="cuda"), drift=True)
    torch.cuda.synchronize()
    return out


def _bounds(sy, r):
    ref = O.evaluate(sy, r, with_intermediates=True)
    L = sy.lam.shape[0]
    gam = (2 * L + 4) * 2.0 ** -24
    nu = sy.n_up
    Phi, G, H, A = ref["Phi"], ref["gradPhi"], ref["lapPhi"], ref["A"]
    gJ = ref["gradJ"]
    Q = H + 2 * (G * gJ.unsqueeze(2)).sum(-1)
    aL = sy.lam.abs()
    absW = Phi[:, :nu].abs() @ aL @ Phi[:, nu:].abs().transpose(1, 2)
    absV = Q[:, :nu].abs() @ aL @ Phi[:, nu:].abs().transpose(1, 2) + \
        Phi[:, :nu].abs() @ aL @ Q[:, nu:].abs().transpose(1, 2)
    V = Q[:, :nu] @ sy.lam @ Phi[:, nu:].transpose(1, 2) + \
        Phi[:, :nu] @ sy.lam @ Q[:, nu:].transpose(1, 2)
    AVA = A @ V @ A
    b_logdet = gam * (A.abs().transpose(1, 2) * absW).sum(dim=(1, 2))
    b_ekin = 0.5 * gam * ((AVA.abs().transpose(1, 2) * absW).sum(dim=(1, 2)) +
                          (A.abs().transpose(1, 2) * absV).sum(dim=(1, 2)))
    return ref, b_logdet, b_ekin


@pytest.mark.parametrize("name", ["tiny", "mol160"])
def test_mixed_eval_within_forward_error_bound(name):
    P = need_gpu()
    if name == "tiny":
        w, idx = C.tiny_3nuc_10e(), list(range(64))
    else:
        w, idx = C.mol_40nuc_160e(n_walkers=64), [0, 9, 31, 50, 63]
    out = _gpu_eval(P, w)
    sy = O.from_workload_system(w.system)
    ref, b_ld, b_ek = _bounds(sy, torch.tensor(w.r0[idx]))
    d_ld = (out["logabs"].cpu()[idx] - ref["logabs"]).abs()
    d_ek = (out["e_kin"].cpu()[idx] - ref["e_kin"]).abs()
    d_el = (out["e_loc"].cpu()[idx] - ref["e_loc"]).abs()
    print(f"[mixed fp32 {name}] max |d logabs| {d_ld.max():.3e} (bound {b_ld.min():.3e}..{b_ld.max():.3e}); "
          f"max |d e_kin| {d_ek.max():.3e} (bound {b_ek.min():.3e}..{b_ek.max():.3e}); "
          f"max rel err logabs {rel_err(out['logabs'].cpu()[idx], ref['logabs']).max():.3e}, "
          f"e_loc {rel_err(out['e_loc'].cpu()[idx], ref['e_loc']).max():.3e}")
    assert torch.all(d_ld <= b_ld + 1e-10)
    assert torch.all(d_ek <= b_ek + 1e-9)
    # the potential is FP64 on both sides: e_loc - e_kin agrees to FP64 rounding
    assert torch.allclose(out["e_loc"].cpu()[idx] - out["e_kin"].cpu()[idx], ref["V"], rtol=1e-12, atol=1e-10)
    assert torch.equal(out["sign"].cpu()[idx], ref["sign"])


@pytest.mark.parametrize("mode", ["mixed", "mixed_bf16"])
@pytest.mark.parametrize("name", ["tiny", "mol160"])
def test_refined_mixed_eval_meets_1e6(name, mode):
    P = need_gpu()
    if name == "tiny":
        w, idx = C.tiny_3nuc_10e(), list(range(64))
    else:
        w, idx = C.mol_40nuc_160e(n_walkers=64), [0, 9, 31, 50, 63]
    out = _gpu_eval(P, w, P.QMC_MIXED if mode == "mixed" else P.QMC_MIXED_BF16)
    ref = O.evaluate(O.from_workload_system(w.system), torch.tensor(w.r0[idx]))
    e_la = rel_err(out["logabs"].cpu()[idx], ref["logabs"]).max().item()
    e_el = rel_err(out["e_loc"].cpu()[idx], ref["e_loc"]).max().item()
    e_dr = ((out["drift"].cpu()[idx] - ref["drift"]).abs().max() / ref["drift"].abs().max()).item()
    print(f"[{mode} refined {name}] max rel err logabs {e_la:.3e}, e_loc {e_el:.3e}, drift {e_dr:.3e}")
    assert e_la <= 1e-6 and e_el <= 1e-6 and e_dr <= 1e-6
    assert torch.equal(out["sign"].cpu()[idx], ref["sign"])


@pytest.mark.parametrize("mode", ["mixed", "mixed_bf16"])
def test_refined_mixed_eval_after_moves(mode):
    # moves run on the reduced-precision copies (P halves rebuilt from them); a
    # later evaluation starts from scratch and is again FP64-accurate
    P = need_gpu()
    w = C.mol_40nuc_160e(n_walkers=32)
    sysh = P.JAGPSystem(w.system, precision=P.QMC_MIXED if mode == "mixed" else P.QMC_MIXED_BF16)
    wk = P.Walkers(sysh, 32)
    wk.eval_batch(torch.tensor(w.r0, device="cuda"))
    d, u = C.chain_arrays(55, 200, 32)
    wk.vmc_steps(0, torch.tensor(d, device="cuda"), torch.tensor(u, device="cuda"))
    r = wk.read(P.STATE_R)
    out = wk.eval_batch(r)
    torch.cuda.synchronize()
    idx = [0, 13, 31]
    rc = r.cpu()
    assert not torch.equal(rc, torch.tensor(w.r0))
    ref = O.evaluate(O.from_workload_system(w.system), rc[idx])
    assert rel_err(out["logabs"].cpu()[idx], ref["logabs"]).max().item() <= 1e-6
    assert rel_err(out["e_loc"].cpu()[idx], ref["e_loc"]).max().item() <= 1e-6


@pytest.mark.parametrize("mode", ["w_fp32", "mixed", "mixed_bf16"])
def test_mixed_moves_ratio_within_bound(mode):
    # QMC_W_FP32: after an FP32 evaluation, the ratio R = w'^T A[:,e] (up) or
    # A[e,:] w' (down) carries two first-order error terms: the FP32 rows of P in
    # w' = P_other psi',  |dw'| <= gamma |Phi_other| |Lambda| |psi'|,  and the
    # inverse of the FP32-built W, dA = -A dW A with
    #   |dW| <= gamma |Phi_up| |Lambda| |Phi_dn|^T,
    # giving |dR| <= |dw'|.|A col| + sum_ik |(w'^T A)_i| |dW_ik| |A_ke| (up; the
    # transpose for down), times exp(dJ).
    # Refined modes: A is FP64-accurate and the stored rows are the FP64 P
    # rounded once, |dP| <= u |P| (u = 2^-24 FP32, 2^-8 BF16), so
    # |dR| <= u (|P_other| |psi'|) . |A col|, times exp(dJ).
    P = need_gpu()
    prec = {"w_fp32": P.QMC_W_FP32, "mixed": P.QMC_MIXED, "mixed_bf16": P.QMC_MIXED_BF16}[mode]
    w = C.mol_40nuc_160e(n_walkers=16)
    sysh = P.JAGPSystem(w.system, precision=prec)
    wk = P.Walkers(sysh, 16)
    r = torch.tensor(w.r0)
    sy = O.from_workload_system(w.system)
    L = sy.lam.shape[0]
    gam = (2 * L + 4) * 2.0 ** -24
    u = 2.0 ** -8 if mode == "mixed_bf16" else 2.0 ** -24
    nu = sy.n_up
    disp = torch.tensor(C.chain_arrays(13, 2, 16)[0])
    ref = O.evaluate(sy, r, with_intermediates=True)
    Phi, A = ref["Phi"], ref["A"]
    absW = Phi[:, :nu].abs() @ sy.lam.abs() @ Phi[:, nu:].abs().transpose(1, 2)
    for t, e in enumerate((3, 120)):
        wk.eval_batch(r.cuda())
        rn = r[:, e] + disp[t]
        ratio = wk.propose(e, rn.cuda().contiguous())
        torch.cuda.synchronize()
        rr = O.move_ratio(sy, r, e, rn)
        psi_n = O.basis(sy, rn)[0]
        if e < nu:
            P_oth = Phi[:, nu:] @ sy.lam.T            # P_dn rows = Phi_dn Lambda^T
            wn = torch.einsum('wjm,wm->wj', P_oth, psi_n)
            col = A[:, :, e]
            if mode == "w_fp32":
                dw = gam * torch.einsum('wm,mn,wjn->wj', psi_n.abs(), sy.lam.abs(), Phi[:, nu:].abs())
                v = torch.einsum('wj,wji->wi', wn, A)
                b = (dw * col.abs()).sum(-1) + gam * torch.einsum('wi,wik,wk->w', v.abs(), absW, col.abs())
            else:
                dw = u * torch.einsum('wjm,wm->wj', P_oth.abs(), psi_n.abs())
                b = (dw * col.abs()).sum(-1)
        else:
            ed = e - nu
            P_oth = Phi[:, :nu] @ sy.lam               # P_up rows = Phi_up Lambda
            wn = torch.einsum('wim,wm->wi', P_oth, psi_n)
            row = A[:, ed, :]
            if mode == "w_fp32":
                dw = gam * torch.einsum('wim,mn,wn->wi', Phi[:, :nu].abs(), sy.lam.abs(), psi_n.abs())
                v = torch.einsum('wli,wi->wl', A, wn)
                b = (dw * row.abs()).sum(-1) + gam * torch.einsum('wk,wkl,wl->w', row.abs(), absW, v.abs())
            else:
                dw = u * torch.einsum('wim,wm->wi', P_oth.abs(), psi_n.abs())
                b = (dw * row.abs()).sum(-1)
        r2 = r.clone(); r2[:, e] = rn
        bound = b * torch.exp(O.jastrow(sy, r2)[0] - ref["J"])
        d = (ratio.cpu() - rr).abs()
        print(f"[{mode} moves e={e}] max |d ratio| {d.max():.3e}, max rel {(d / rr.abs()).max():.3e}, "
              f"bound {bound.min():.3e}..{bound.max():.3e}")
        assert torch.all(d <= bound * (1 + 1e-6) + 1e-12)


@pytest.mark.parametrize("precision", ["mixed", "mixed_bf16", "fp32"])
def test_set_params_equals_fresh_system(precision):
    # device parameter updates refresh the reduced-precision copies (Lambda's
    # FP32 copy, the basis packing, the Jastrow scalars): evaluations and a
    # chain equal those of a system created with the new parameters, bitwise
    P = need_gpu()
    prec = {"mixed": P.QMC_MIXED, "mixed_bf16": P.QMC_MIXED_BF16, "fp32": P.QMC_W_FP32}[precision]
    w = C.tiny_3nuc_10e(n_walkers=16, n_steps=60)
    s = w.system
    rng = np.random.default_rng(8)
    L_ = len(s.lam)
    a = rng.standard_normal((L_, L_))
    lam2 = s.lam + 0.01 * (a + a.T) / L_
    R2 = s.R + 0.03 * rng.standard_normal(s.R.shape)
    z2 = s.zeta * 1.02
    jas2 = np.concatenate([np.asarray(s.j1_b) * 1.1, np.asarray(s.j2) * 0.9])
    T = lambda x: torch.tensor(np.ascontiguousarray(x), device="cuda")
    upd = P.JAGPSystem(s, precision=prec)
    upd.set_params(R=T(R2), zeta=T(z2), lam=T(lam2), jas=T(jas2))
    fresh = P.JAGPSystem(dataclasses.replace(s, R=R2, zeta=z2, lam=lam2, j1_b=jas2[:len(s.Z)],
                                             j2=jas2[len(s.Z):]), precision=prec)
    r = torch.tensor(w.r0, device="cuda")
    wa, wb = P.Walkers(upd, 16), P.Walkers(fresh, 16)
    oa, ob = wa.eval_batch(r), wb.eval_batch(r)
    d, u = torch.tensor(w.disp, device="cuda"), torch.tensor(w.unif, device="cuda")
    wa.vmc_steps(0, d, u)
    wb.vmc_steps(0, d, u)
    torch.cuda.synchronize()
    for k in ("logabs", "e_loc", "drift"):
        assert torch.equal(oa[k], ob[k]), k
    assert torch.equal(wa.read(P.STATE_R), wb.read(P.STATE_R))
    assert torch.equal(wa.read(P.STATE_LOGABS), wb.read(P.STATE_LOGABS))
