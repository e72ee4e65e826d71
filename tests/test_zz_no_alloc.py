"""qmc_sr_step_static, the allocation-free SR step, through the raw C ABI.

It must give what qmc_sr_step gives with a caller workspace (the same kernels
in the same order: bitwise equal), on two calls in a row whose second input is
smaller (the static array keeps the first call's contents; nothing in it may
leak into the second), agree with the oracle's direct solve (Stochastic
reconfiguration section: (S + eps diag S) delta = f; bars as the SR parity
test), and refuse a problem beyond its 16 MiB array before enqueuing anything.
"""
import ctypes

import pytest
import torch

from gpu_util import need_gpu
from oracle import estimators as E

pytestmark = pytest.mark.gpu


def _inputs(M, Pn, seed, weighted):
    g = torch.Generator().manual_seed(seed)
    B = torch.randn(Pn, Pn, generator=g, dtype=torch.float64) / Pn ** 0.5 + torch.eye(Pn, dtype=torch.float64)
    Ok = torch.randn(M, Pn, generator=g, dtype=torch.float64) @ B
    Ok = Ok * torch.logspace(-1, 1, Pn, dtype=torch.float64) + 0.3
    el = -5.0 + torch.randn(M, generator=g, dtype=torch.float64) + 0.5 * Ok[:, 0]
    wts = 0.5 + torch.rand(M, generator=g, dtype=torch.float64) if weighted else None
    return Ok, el, wts


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _static(lib, Ok, el, wts, eps, max_iter, tol):
    M, Pn = Ok.shape
    dev = Ok.device
    delta = torch.full((Pn,), float("nan"), dtype=torch.float64, device=dev)
    f = torch.full((Pn,), float("nan"), dtype=torch.float64, device=dev)
    res = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.qmc_sr_step_static(M, Pn, _p(Ok), _p(el), _p(wts), eps, max_iter, tol, _p(delta), _p(f), _p(res), st)
    assert rc == 0, lib.qmc_last_error().decode()
    return delta, f, res


def _with_workspace(lib, Ok, el, wts, eps, max_iter, tol):
    M, Pn = Ok.shape
    dev = Ok.device
    nb = lib.qmc_sr_workspace_size(M, Pn)
    work = torch.full(((nb + 7) // 8,), float("nan"), dtype=torch.float64, device=dev)
    delta = torch.empty(Pn, dtype=torch.float64, device=dev)
    f = torch.empty(Pn, dtype=torch.float64, device=dev)
    res = torch.empty(1, dtype=torch.float64, device=dev)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.qmc_sr_step(M, Pn, _p(Ok), _p(el), _p(wts), eps, max_iter, tol, _p(delta), _p(f), _p(res),
                         _p(work), work.numel() * 8, st)
    assert rc == 0, lib.qmc_last_error().decode()
    return delta, f, res


def test_static_sr_step_equals_workspace_sr_step_twice():
    need_gpu()
    from paper_2002_07401_amd import binding as B
    lib = B.load()
    eps = 1e-3
    # first a larger problem, then a smaller one in the same static array
    for (M, Pn, weighted, seed) in ((1000, 513, True, 41), (200, 50, False, 42)):
        Ok, el, wts = _inputs(M, Pn, seed, weighted)
        cu = lambda t: None if t is None else t.cuda()
        Ok_d, el_d, w_d = cu(Ok), cu(el), cu(wts)
        a = _static(lib, Ok_d, el_d, w_d, eps, 4 * Pn + 20, 1e-14)
        b = _with_workspace(lib, Ok_d, el_d, w_d, eps, 4 * Pn + 20, 1e-14)
        torch.cuda.synchronize()
        for x, y, name in zip(a, b, ("delta", "force", "residual")):
            assert torch.equal(x, y), (M, Pn, name)
        d_ref, f_ref, _ = E.sr_step(Ok, el, eps, wts)
        ef = ((a[1].cpu() - f_ref).abs().max() / f_ref.abs().max()).item()
        ed = ((a[0].cpu() - d_ref).abs().max() / d_ref.abs().max()).item()
        print(f"[sr static M={M} P={Pn}] f {ef:.3e} delta {ed:.3e} residual {a[2].item():.3e}")
        assert ef <= 1e-12 and ed <= 1e-9 and a[2].item() <= 1e-13


def test_static_sr_step_refuses_problems_beyond_its_array():
    need_gpu()
    from paper_2002_07401_amd import binding as B
    lib = B.load()
    M, Pn = 4096, 40000        # qmc_sr_workspace_size > 16 MiB
    assert lib.qmc_sr_workspace_size(M, Pn) > 16 * 1024 * 1024
    dummy = torch.zeros(8, dtype=torch.float64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.qmc_sr_step_static(M, Pn, _p(dummy), _p(dummy), None, 1e-3, 10, 1e-12, _p(dummy), None, None, st)
    assert rc == -2
    assert "16 MiB" in lib.qmc_last_error().decode()
