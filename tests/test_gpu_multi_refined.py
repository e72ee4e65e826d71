"""QMC_REFINED members in one multi-system launch per phase: the screened
streams run per walker inside the persistent rows phase (the blocked stream
where its LDS layout allows, else the plain one), the P rebuilds are the int8
digit products with their transposed rows and column maxima.

* Each member (the eight sizes 16-256 e- of the uneven-systems workload, and a
  polarized member beside them) evolves as it does alone: positions, log|Psi|,
  sign, W and W^{-1} bitwise equal to qmc_vmc_steps with the same draws.
* The small members' chains equal the oracle's chains (positions bitwise),
  log|Psi| within 1e-8.
* A captured graph reproduces the direct launches bitwise.
"""
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu

SIZES = (16, 32, 48, 64, 96, 128, 192, 256)


def _members(P, Wk, polarized=False):
    out = []
    ws = [C.multi_system(n, n_walkers=Wk) for n in SIZES]
    if polarized:
        ws.append(C.polarized_4nuc_20e(n_walkers=Wk))
    for w in ws:
        sysh = P.JAGPSystem(w.system, precision=P.QMC_REFINED)
        wk = P.Walkers(sysh, Wk, adjoint=False)
        wk.eval_batch(torch.tensor(w.r0[:Wk], device="cuda"))
        out.append((w, sysh, wk))
    return out


def test_multi_refined_members_equal_single_runs():
    P = need_gpu()
    Wk, n_steps = 8, 100
    grp = _members(P, Wk, polarized=True)
    solo = _members(P, Wk, polarized=True)
    draws = [C.chain_arrays(1700 + k, n_steps, Wk) for k in range(len(grp))]
    disp = [torch.tensor(d, device="cuda") for d, _ in draws]
    unif = [torch.tensor(u, device="cuda") for _, u in draws]
    m = P.MultiSystem([wk for _, _, wk in grp])
    m.vmc_steps(n_steps, disp, unif)
    for k, (_, _, wk) in enumerate(solo):
        wk.vmc_steps(0, disp[k], unif[k])
    torch.cuda.synchronize()
    for k in range(len(grp)):
        a, b = grp[k][2], solo[k][2]
        for item in (P.STATE_R, P.STATE_LOGABS, P.STATE_SIGN, P.STATE_AINV, P.STATE_W):
            assert torch.equal(a.read(item), b.read(item)), (grp[k][0].system.name, item)
    m.close()


def test_multi_refined_chains_match_oracle():
    P = need_gpu()
    Wk, n_steps = 4, 40
    grp = _members(P, Wk)
    draws = [C.chain_arrays(1900 + k, n_steps, Wk) for k in range(len(SIZES))]
    m = P.MultiSystem([wk for _, _, wk in grp])
    m.vmc_steps(n_steps, [torch.tensor(d, device="cuda") for d, _ in draws],
                [torch.tensor(u, device="cuda") for _, u in draws])
    torch.cuda.synchronize()
    for k, n in enumerate(SIZES[:4]):
        w, _, wk = grp[k]
        sy = O.from_workload_system(w.system)
        rf, _, _ = O.run_chain(sy, torch.tensor(w.r0[:Wk]), torch.tensor(draws[k][0]), torch.tensor(draws[k][1]))
        assert torch.equal(wk.read(P.STATE_R).cpu(), rf), n
        assert rel_err(wk.read(P.STATE_LOGABS).cpu(), O.log_psi(sy, rf)[0]).max().item() <= 1e-8, n
    m.close()


def test_multi_refined_graph_replay_equals_direct_launches():
    P = need_gpu()
    Wk, n_steps = 8, 768
    ga = _members(P, Wk)
    gb = _members(P, Wk)
    ma = P.MultiSystem([wk for _, _, wk in ga])
    mb = P.MultiSystem([wk for _, _, wk in gb])
    for _ in range(2):           # the second call replays the captured graph
        ma.vmc_steps(n_steps, seed=83, sigma=0.3, use_graph=True)
        mb.vmc_steps(n_steps, seed=83, sigma=0.3, use_graph=False)
    torch.cuda.synchronize()
    moved = 0
    for k in range(len(SIZES)):
        ra, rb = ga[k][2].read(P.STATE_R), gb[k][2].read(P.STATE_R)
        assert torch.equal(ra, rb)
        assert torch.equal(ga[k][2].read(P.STATE_LOGABS), gb[k][2].read(P.STATE_LOGABS))
        moved += int((ra.cpu() != torch.tensor(ga[k][0].r0[:Wk])).any(-1).sum())
    assert moved > 0
    ma.close(); mb.close()
