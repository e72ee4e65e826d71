"""Several systems of uneven electron count moved by one persistent launch per
phase (qmc_multi_vmc_steps), optionally captured in a HIP graph.

* Each member must evolve exactly as it does alone (qmc_vmc_steps with the same
  displacements and uniforms): positions, log|Psi| and W^{-1} bitwise equal.
* The device Philox4x32-10 draws must equal the oracle's generator (uniforms
  bitwise; Box-Muller normals to 1e-15, the two libms differing by ulps).
* A graph replay must reproduce the direct launches bitwise.
"""
import numpy as np
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from oracle import philox as PH
from workloads import configs as C

pytestmark = pytest.mark.gpu

SIZES = (16, 32, 48, 64, 96, 128, 192, 256)   # every member size of the 8-system workload


def _members(P, Wk, precision=None):
    out = []
    for n in SIZES:
        w = C.multi_system(n, n_walkers=Wk)
        sysh = P.JAGPSystem(w.system) if precision is None else P.JAGPSystem(w.system, precision=precision)
        wk = P.Walkers(sysh, Wk)
        wk.eval_batch(torch.tensor(w.r0, device="cuda"))
        out.append((w, sysh, wk))
    return out


def test_philox_draws_match_oracle_generator():
    P = need_gpu()
    for member, step in ((0, 0), (3, 12345), (7, 2 ** 33 + 5)):
        d, u = P.philox_draws(2002, member, 300, step, 0.3)
        torch.cuda.synchronize()
        dr, ur = PH.metropolis_draws(2002, member, np.arange(300), step, 0.3)
        assert np.array_equal(u.cpu().numpy(), ur)
        assert np.abs(d.cpu().numpy() - dr).max() <= 1e-15


def test_multi_explicit_draws_equal_single_runs():
    P = need_gpu()
    Wk, n_steps = 8, 100
    grp = _members(P, Wk)
    solo = _members(P, Wk)
    draws = [C.chain_arrays(700 + k, n_steps, Wk) for k in range(len(SIZES))]
    disp = [torch.tensor(d, device="cuda") for d, _ in draws]
    unif = [torch.tensor(u, device="cuda") for _, u in draws]
    m = P.MultiSystem([wk for _, _, wk in grp])
    m.vmc_steps(n_steps, disp, unif)
    for k, (_, _, wk) in enumerate(solo):
        wk.vmc_steps(0, disp[k], unif[k])
    torch.cuda.synchronize()
    for k, n in enumerate(SIZES):
        a, b = grp[k][2], solo[k][2]
        for item in (P.STATE_R, P.STATE_LOGABS, P.STATE_SIGN, P.STATE_AINV, P.STATE_W):
            assert torch.equal(a.read(item), b.read(item)), (n, item)
    m.close()


def test_multi_chain_matches_oracle_for_small_members():
    P = need_gpu()
    Wk, n_steps = 4, 40
    grp = _members(P, Wk)
    draws = [C.chain_arrays(900 + k, n_steps, Wk) for k in range(len(SIZES))]
    m = P.MultiSystem([wk for _, _, wk in grp])
    m.vmc_steps(n_steps, [torch.tensor(d, device="cuda") for d, _ in draws],
                [torch.tensor(u, device="cuda") for _, u in draws])
    torch.cuda.synchronize()
    for k, n in enumerate(SIZES[:4]):
        w, _, wk = grp[k]
        sy = O.from_workload_system(w.system)
        rf, _, _ = O.run_chain(sy, torch.tensor(w.r0), torch.tensor(draws[k][0]), torch.tensor(draws[k][1]))
        assert torch.equal(wk.read(P.STATE_R).cpu(), rf)
        assert rel_err(wk.read(P.STATE_LOGABS).cpu(), O.log_psi(sy, rf)[0]).max().item() <= 1e-10
    m.close()


def test_multi_graph_replay_equals_direct_launches():
    P = need_gpu()
    Wk, n_steps = 8, 768         # 768 = lcm of (N, refresh period) over the members: the second call replays
    ga = _members(P, Wk)
    gb = _members(P, Wk)
    ma = P.MultiSystem([wk for _, _, wk in ga])
    mb = P.MultiSystem([wk for _, _, wk in gb])
    for _ in range(2):           # second call replays the captured graph
        ma.vmc_steps(n_steps, seed=77, sigma=0.3, use_graph=True)
        mb.vmc_steps(n_steps, seed=77, sigma=0.3, use_graph=False)
    torch.cuda.synchronize()
    moved = 0
    for k in range(len(SIZES)):
        ra, rb = ga[k][2].read(P.STATE_R), gb[k][2].read(P.STATE_R)
        assert torch.equal(ra, rb)
        assert torch.equal(ga[k][2].read(P.STATE_LOGABS), gb[k][2].read(P.STATE_LOGABS))
        moved += int((ra.cpu() != torch.tensor(ga[k][0].r0)).any(-1).sum())
    assert moved > 0
    ma.close(); mb.close()


def test_multi_philox_chain_equals_single_with_same_draws():
    P = need_gpu()
    Wk, n_steps, seed = 8, 50, 4242
    grp = _members(P, Wk)
    solo = _members(P, Wk)
    m = P.MultiSystem([wk for _, _, wk in grp])
    m.vmc_steps(n_steps, seed=seed, sigma=0.3)
    for k, (_, _, wk) in enumerate(solo):
        for t in range(n_steps):
            d, u = P.philox_draws(seed, k, Wk, t, 0.3)
            wk.vmc_steps(t, d.view(1, Wk, 3).contiguous(), u.view(1, Wk).contiguous())
    torch.cuda.synchronize()
    for k in range(len(SIZES)):
        assert torch.equal(grp[k][2].read(P.STATE_R), solo[k][2].read(P.STATE_R))
    m.close()


def test_multi_autotune_then_steps_stay_correct():
    P = need_gpu()
    Wk, n_steps = 8, 64
    grp = _members(P, Wk)
    m = P.MultiSystem([wk for _, _, wk in grp])
    rows, grid = m.autotune()
    assert rows in (8, 16, 32) and grid > 0
    m.vmc_steps(n_steps, seed=5, sigma=0.3)
    torch.cuda.synchronize()
    for k in range(2):
        w, _, wk = grp[k]
        sy = O.from_workload_system(w.system)
        r = wk.read(P.STATE_R).cpu()
        assert rel_err(wk.read(P.STATE_LOGABS).cpu(), O.log_psi(sy, r)[0]).max().item() <= 1e-10
    m.close()


@pytest.mark.parametrize("precision", ["fp32", "mixed", "mixed_bf16"])
def test_multi_reduced_precision_members_equal_single_runs(precision):
    # FP32 / BF16 rows in the persistent launches: each member's chain equals
    # the single-system run of the same storage type on the same draws
    P = need_gpu()
    prec = {"fp32": P.QMC_W_FP32, "mixed": P.QMC_MIXED, "mixed_bf16": P.QMC_MIXED_BF16}[precision]
    Wk, n_steps = 8, 100
    grp = _members(P, Wk, prec)
    solo = _members(P, Wk, prec)
    draws = [C.chain_arrays(730 + k, n_steps, Wk) for k in range(len(SIZES))]
    disp = [torch.tensor(d, device="cuda") for d, _ in draws]
    unif = [torch.tensor(u, device="cuda") for _, u in draws]
    m = P.MultiSystem([wk for _, _, wk in grp])
    m.vmc_steps(n_steps, disp, unif)
    for k, (_, _, wk) in enumerate(solo):
        wk.vmc_steps(0, disp[k], unif[k])
    torch.cuda.synchronize()
    for k, n in enumerate(SIZES):
        a, b = grp[k][2], solo[k][2]
        assert torch.equal(a.read(P.STATE_R), b.read(P.STATE_R)), (precision, n)
        la, lb = a.read(P.STATE_LOGABS).cpu(), b.read(P.STATE_LOGABS).cpu()
        assert rel_err(la, lb).max().item() <= 1e-12, (precision, n)
    # the FP64 log|Psi| carried through the chain against the oracle (small members)
    if precision == "mixed":
        for k in range(2):
            w, _, wk = grp[k]
            sy = O.from_workload_system(w.system)
            r = wk.read(P.STATE_R).cpu()
            assert rel_err(wk.read(P.STATE_LOGABS).cpu(), O.log_psi(sy, r)[0]).max().item() <= 1e-6
    m.close()
