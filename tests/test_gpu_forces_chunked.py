"""The walker-summed adjoint (qmc_forces, per_walker = 0) at walker counts that
run its chunked reductions: the Lambda and unpaired-orbital gradients are
summed over chunks of ceil(Wk / 64) walkers with a shorter last chunk when
64 does not divide Wk.

Every summed output is compared with (a) the host sum of the same call's
per-walker outputs (same arithmetic per walker, different summation order:
1e-12 of scale) and (b) the oracle's reverse-mode gradient of
sum_w (gl[w] log|Psi_w| + ge[w] e_L,w) (Derivatives of energy section; bar
1e-8 of scale, as the other adjoint tests).
"""
import dataclasses

import numpy as np
import pytest
import torch

from gpu_util import need_gpu
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu

KEYS = ("R", "zeta", "lam", "jas", "r")


def _scale_err(a, b):
    return (a - b).abs().max().item() / max(1.0, b.abs().max().item())


def _oracle_unpaired_grads(sy, r, gl, ge):
    U = sy.unpaired.detach().clone().requires_grad_(True)
    out = O.evaluate(dataclasses.replace(sy, unpaired=U), r)
    F = (gl * out["logabs"]).sum() + (ge * out["e_loc"]).sum()
    return torch.autograd.grad(F, U)[0]


def _run(P, w, Wk, seed, with_unpaired=False, oracle=True):
    sysh = P.JAGPSystem(w.system)
    wk = P.Walkers(sysh, Wk)
    r = torch.tensor(w.r0[:Wk])
    rng = np.random.default_rng(seed)
    gl = torch.tensor(rng.normal(size=Wk))
    ge = torch.tensor(rng.normal(size=Wk))
    summed = wk.forces(r.cuda(), gl.cuda(), ge.cuda())
    per = wk.forces(r.cuda(), gl.cuda(), ge.cuda(), per_walker=True)
    torch.cuda.synchronize()
    keys = KEYS + (("unpaired",) if with_unpaired else ())
    for k in keys:
        a = summed[k].cpu()
        b = per[k].cpu() if k == "r" else per[k].cpu().sum(0)
        err = _scale_err(a, b)
        print(f"[forces Wk={Wk}] {k}: summed vs host sum of per-walker {err:.3e}")
        assert err <= 1e-12, (Wk, k, err)
    if oracle:
        sy = O.from_workload_system(w.system)
        ref = O.forces_vjp(sy, r, gl, ge)
        if with_unpaired:
            ref["unpaired"] = _oracle_unpaired_grads(sy, r, gl, ge)
        for k in keys:
            err = _scale_err(summed[k].cpu(), ref[k])
            print(f"[forces Wk={Wk}] {k}: summed vs oracle {err:.3e}")
            assert err <= 1e-8, (Wk, k, err)


def test_forces_sum_two_walker_chunks_with_remainder():
    # Wk = 65: chunks of 2 walkers, 32 full chunks and a last chunk of 1
    P = need_gpu()
    _run(P, C.tiny_3nuc_10e(n_walkers=65), 65, 11)


def test_forces_sum_unpaired_orbitals_chunked():
    # Wk = 67: chunks of 2, 33 full chunks and a last chunk of 1; the
    # unpaired-orbital gradients take the same chunked path
    P = need_gpu()
    _run(P, C.polarized_4nuc_20e(n_walkers=67), 67, 12, with_unpaired=True)


def test_forces_sum_80e_512_walkers():
    # the 80-electron forces workload at its full 512 walkers: chunks of 8
    P = need_gpu()
    _run(P, C.forces_20nuc_80e(n_walkers=512), 512, 13)


def test_forces_sum_80e_uneven_chunks():
    # 515 walkers: chunks of 9, 57 full chunks and a last chunk of 2
    P = need_gpu()
    _run(P, C.forces_20nuc_80e(n_walkers=515), 515, 14, oracle=False)
