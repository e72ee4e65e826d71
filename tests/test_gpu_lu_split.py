"""The column-split Gauss-Jordan inverse (64 < n <= 88: two waves, each with
the columns of one half of W for every row, the pivot row taken by readlane
from the wave's own registers).

On the uneven-batch members with n = 65, 72, 80 and 88 electrons per spin
(W padded to 72, 72, 80 and 88 rows):

* evaluation against the oracle at the FP64 bar (relative 1e-10 on log|Psi|
  and E_loc, 1e-8 on the drift) and the sign;
* the inverse against the inverse of the exported W (numpy, FP64): relative
  1e-9 of its largest entry, and |W A - I| below 1e-9;
* 40 Metropolis steps (a refresh after 32 moves of one spin): the tracked
  log|Psi| and inverse equal those of a fresh evaluation at the final
  positions;
* W = 0 (Lambda = 0) is reported singular (status 1, log|Psi| = -inf).
"""
import dataclasses

import numpy as np
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu

WK = 6


def _eval(P, w, r=None):
    sysh = P.JAGPSystem(w.system)
    wk = P.Walkers(sysh, WK)
    r = torch.tensor(w.r0[:WK], device="cuda") if r is None else r
    out = wk.eval_batch(r, drift=True)
    torch.cuda.synchronize()
    return sysh, wk, out


@pytest.mark.parametrize("n_elec", [130, 144, 160, 176])
def test_split_inverse_eval_inverse_and_refresh(n_elec):
    P = need_gpu()
    w = C.multi_system(n_elec, n_walkers=WK)
    sysh, wk, out = _eval(P, w)
    ref = O.evaluate(O.from_workload_system(w.system), torch.tensor(w.r0[:WK]))
    for k in ("logabs", "e_loc"):
        assert rel_err(out[k].cpu(), ref[k]).max().item() <= 1e-10, k
    d = out["drift"].cpu()
    assert ((d - ref["drift"]).abs() / ref["drift"].abs().clamp(min=1.0)).max().item() <= 1e-8
    assert torch.equal(out["sign"].cpu(), ref["sign"])
    assert (out["status"].cpu() == 0).all()
    Wm = wk.read(P.STATE_W).cpu().numpy()
    A = wk.read(P.STATE_AINV).cpu().numpy()
    torch.cuda.synchronize()
    n = n_elec // 2
    for i in range(WK):
        Ai = np.linalg.inv(Wm[i])
        assert np.abs(A[i] - Ai).max() <= 1e-9 * np.abs(Ai).max()
        assert np.abs(Wm[i] @ A[i] - np.eye(n)).max() <= 1e-9
    dd, uu = C.chain_arrays(23, 40, WK)
    wk.vmc_steps(0, torch.tensor(dd, device="cuda"), torch.tensor(uu, device="cuda"))
    r = wk.read(P.STATE_R)
    la, A1 = wk.read(P.STATE_LOGABS), wk.read(P.STATE_AINV)
    _, wk2, out2 = _eval(P, w, r=r)
    assert rel_err(la.cpu(), out2["logabs"].cpu()).max().item() <= 1e-10
    A2 = wk2.read(P.STATE_AINV)
    assert ((A1 - A2).abs().max() / A2.abs().max()).item() <= 1e-8


def test_split_inverse_singular_status():
    P = need_gpu()
    w = C.multi_system(160, n_walkers=WK)
    zero = dataclasses.replace(w.system, lam=np.zeros_like(w.system.lam))
    _, _, out = _eval(P, dataclasses.replace(w, system=zero))
    assert (out["status"].cpu() == 1).all()
    assert torch.isinf(out["logabs"].cpu()).all()
