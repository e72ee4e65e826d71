"""ctypes binding of libqmc_jagp.so (include/qmc.h).

Argument marshalling only: every step of the wave-function path runs in the
HIP kernels of the library.  PyTorch supplies device memory and the stream.
Importing this module does not load the library; the first use does, and it
raises QMCError when the library is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqmc_jagp.so")

QMC_FP64 = 0
QMC_W_FP32 = 1
QMC_MIXED = 2
QMC_MIXED_BF16 = 3
QMC_W_BF16 = 4
QMC_W_FP8 = 5
QMC_REFINED = 6

WALKERS_ADJOINT = 1

STATE_R, STATE_LOGABS, STATE_SIGN, STATE_W, STATE_AINV, STATE_PHI, STATE_RESIDUAL, STATE_KEPT = range(8)

STATUS_NAMES = {0: "OK", -1: "ERR_ARG", -2: "ERR_SHAPE", -3: "ERR_HIP", -4: "ERR_OOM",
                -5: "ERR_UNSUPPORTED", -6: "ERR_STATE"}

FUNCTIONS = (
    "qmc_abi_version", "qmc_last_error", "qmc_system_create", "qmc_system_destroy",
    "qmc_walkers_create", "qmc_walkers_destroy", "qmc_eval_batch", "qmc_propose_move",
    "qmc_accept_move", "qmc_vmc_steps", "qmc_walkers_read", "qmc_walkers_set_timing",
    "qmc_walkers_timing", "qmc_forces", "qmc_system_set_params", "qmc_multi_create",
    "qmc_multi_destroy", "qmc_multi_autotune", "qmc_multi_vmc_steps", "qmc_philox_draws",
    "qmc_lrdmc_hops", "qmc_lrdmc_advance", "qmc_walkers_set_timing_mask", "qmc_swct", "qmc_reweight",
    "qmc_sr_workspace_size", "qmc_sr_step", "qmc_jastrow_basis_logderiv", "qmc_pfaffian_logderiv",
    "qmc_system_set_jastrow_basis", "qmc_system_set_pfaffian", "qmc_workspace_size", "qmc_walkers_set_drift_tol",
    "qmc_sr_step_static",
)

TIMER_NAMES = ("basis", "P_build", "W_build", "LU", "Y_build", "rowdot", "assemble", "propose",
               "accept", "other", "propose_prep", "lrdmc_hops", "lrdmc_step", "P_rebuild", "sweep")

# per-walker terms of qmc_lrdmc_hops
LR_TERMS = ("e_loc", "e_kin", "lap_a", "va_shift", "v_sf", "escape", "hfn_diag")


class QMCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Grads(ctypes.Structure):
    _fields_ = [("dR", ctypes.c_void_p), ("dzeta", ctypes.c_void_p), ("dlambda", ctypes.c_void_p),
                ("djas", ctypes.c_void_p), ("dr", ctypes.c_void_p), ("dj1_inh", ctypes.c_void_p),
                ("dj3", ctypes.c_void_p), ("djb_zeta", ctypes.c_void_p), ("dunpaired", ctypes.c_void_p),
                ("dcon_coef", ctypes.c_void_p), ("dpf_uu", ctypes.c_void_p), ("dpf_dd", ctypes.c_void_p),
                ("dunpaired_dn", ctypes.c_void_p)]


class LrdmcParams(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("a_valence", ctypes.c_double), ("tf_scale", ctypes.c_double),
                ("gamma", ctypes.c_double)]


class SystemDesc(ctypes.Structure):
    _fields_ = [
        ("n_nuc", ctypes.c_int32), ("R", ctypes.c_void_p), ("Z", ctypes.c_void_p),
        ("n_basis", ctypes.c_int32), ("center", ctypes.c_void_p), ("l", ctypes.c_void_p),
        ("m", ctypes.c_void_p), ("radial", ctypes.c_void_p), ("zeta", ctypes.c_void_p),
        ("lambda_", ctypes.c_void_p), ("n_up", ctypes.c_int32), ("n_dn", ctypes.c_int32),
        ("j1_form", ctypes.c_int32), ("j1_b", ctypes.c_void_p), ("j2_form", ctypes.c_int32),
        ("n_j2", ctypes.c_int32), ("j2", ctypes.c_void_p), ("precision", ctypes.c_int32),
        ("refresh_every", ctypes.c_int32),
        ("n_jbasis", ctypes.c_int32), ("jb_center", ctypes.c_void_p), ("jb_l", ctypes.c_void_p),
        ("jb_m", ctypes.c_void_p), ("jb_radial", ctypes.c_void_p), ("jb_zeta", ctypes.c_void_p),
        ("j1_inh", ctypes.c_void_p), ("j3", ctypes.c_void_p),
        ("n_contracted", ctypes.c_int32), ("con_ptr", ctypes.c_void_p), ("con_idx", ctypes.c_void_p),
        ("con_coef", ctypes.c_void_p), ("unpaired", ctypes.c_void_p),
        ("pairing", ctypes.c_int32), ("pf_uu", ctypes.c_void_p), ("pf_dd", ctypes.c_void_p),
        ("pf_k", ctypes.c_int32), ("pf_unpaired_dn", ctypes.c_void_p),
    ]


_lib: Optional[ctypes.CDLL] = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the library once; raise QMCError if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise QMCError(-5, f"{path} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, i32, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p
    lib.qmc_abi_version.restype = i32
    lib.qmc_last_error.restype = ctypes.c_char_p
    for name in FUNCTIONS[2:]:
        getattr(lib, name).restype = ctypes.c_int
    lib.qmc_system_create.argtypes = [ctypes.POINTER(SystemDesc), ctypes.POINTER(vp)]
    lib.qmc_system_destroy.argtypes = [vp]
    lib.qmc_walkers_create.argtypes = [vp, i32, i32, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    lib.qmc_workspace_size.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.qmc_walkers_set_drift_tol.argtypes = [vp, ctypes.c_double]
    lib.qmc_walkers_destroy.argtypes = [vp]
    lib.qmc_eval_batch.argtypes = [vp, vp, dp, dp, dp, dp, dp, dp, vp, vp]
    lib.qmc_propose_move.argtypes = [vp, vp, i32, dp, dp, dp, vp]
    lib.qmc_accept_move.argtypes = [vp, vp, i32, vp, vp, vp]
    lib.qmc_vmc_steps.argtypes = [vp, vp, i32, i32, dp, dp, vp, vp]
    lib.qmc_walkers_read.argtypes = [vp, i32, dp, vp]
    lib.qmc_walkers_set_timing.argtypes = [vp, i32]
    lib.qmc_walkers_set_timing_mask.argtypes = [vp, ctypes.c_uint32]
    lib.qmc_walkers_timing.argtypes = [vp, vp, vp]
    lib.qmc_forces.argtypes = [vp, vp, dp, i32, dp, dp, ctypes.POINTER(Grads), vp]
    lib.qmc_system_set_params.argtypes = [vp, dp, dp, dp, dp, vp]
    lib.qmc_multi_create.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp)]
    lib.qmc_multi_destroy.argtypes = [vp]
    lib.qmc_multi_autotune.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), vp]
    lib.qmc_multi_vmc_steps.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_uint64,
                                        ctypes.c_double, i32, vp]
    lib.qmc_philox_draws.argtypes = [ctypes.c_uint64, i32, i32, ctypes.c_uint64, ctypes.c_double, dp, dp, vp]
    lib.qmc_lrdmc_hops.argtypes = [vp, vp, ctypes.POINTER(LrdmcParams), dp, dp, vp]
    lib.qmc_lrdmc_advance.argtypes = [vp, vp, dp, dp, dp, dp, vp, vp]
    lib.qmc_swct.argtypes = [vp, i32, dp, dp, dp, i32, dp, vp]
    lib.qmc_jastrow_basis_logderiv.argtypes = [vp, vp, dp, dp, vp]
    lib.qmc_pfaffian_logderiv.argtypes = [vp, vp, dp, dp, dp, dp, dp, vp]
    lib.qmc_system_set_jastrow_basis.argtypes = [vp, dp, dp, dp, vp]
    lib.qmc_system_set_pfaffian.argtypes = [vp, dp, dp, dp, dp, vp]
    lib.qmc_reweight.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double, dp, dp, vp]
    lib.qmc_sr_workspace_size.restype = ctypes.c_size_t
    lib.qmc_sr_workspace_size.argtypes = [i32, ctypes.c_int64]
    lib.qmc_sr_step.argtypes = [i32, ctypes.c_int64, dp, dp, dp, ctypes.c_double, i32, ctypes.c_double, dp, dp,
                                dp, vp, ctypes.c_size_t, vp]
    lib.qmc_sr_step_static.argtypes = [i32, ctypes.c_int64, dp, dp, dp, ctypes.c_double, i32, ctypes.c_double, dp,
                                       dp, dp, vp]
    _lib = lib
    return lib


def _check(code):
    if code != 0:
        raise QMCError(code, load().qmc_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise QMCError(-1, "device tensor expected")
    if not t.is_contiguous():
        raise QMCError(-1, "contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class JAGPSystem:
    """A system on the current GPU, built from a workloads.System."""

    def __init__(self, s, precision: int = QMC_FP64, refresh_every: Optional[int] = None):
        lib = load()
        self.s = s
        keep = dict(
            R=np.ascontiguousarray(s.R, np.float64), Z=np.ascontiguousarray(s.Z, np.float64),
            center=np.ascontiguousarray(s.center, np.int32), l=np.ascontiguousarray(s.l, np.int32),
            m=np.ascontiguousarray(s.m, np.int32), radial=np.ascontiguousarray(s.radial, np.int32),
            zeta=np.ascontiguousarray(s.zeta, np.float64), lam=np.ascontiguousarray(s.lam, np.float64),
            j1_b=np.ascontiguousarray(s.j1_b, np.float64), j2=np.ascontiguousarray(s.j2, np.float64),
            unpaired=np.ascontiguousarray(np.asarray(s.unpaired, np.float64).reshape(len(s.lam), -1)))
        LJ = 0 if getattr(s, "jb_zeta", None) is None else len(s.jb_zeta)
        if LJ:
            keep.update(jb_center=np.ascontiguousarray(s.jb_center, np.int32),
                        jb_l=np.ascontiguousarray(s.jb_l, np.int32), jb_m=np.ascontiguousarray(s.jb_m, np.int32),
                        jb_radial=np.ascontiguousarray(s.jb_radial, np.int32),
                        jb_zeta=np.ascontiguousarray(s.jb_zeta, np.float64),
                        j1_inh=np.ascontiguousarray(s.j1_inh, np.float64),
                        j3=np.ascontiguousarray(s.j3, np.float64))
        pf = int(getattr(s, "pairing", 0) or 0)
        k_pf = keep["unpaired"].shape[1] if pf else 0
        if pf:
            keep.update(pf_uu=np.ascontiguousarray(s.pf_uu, np.float64), pf_dd=np.ascontiguousarray(s.pf_dd, np.float64),
                        pf_dn=np.ascontiguousarray(np.asarray(s.unpaired_dn, np.float64).reshape(len(s.lam), -1)))
        Cm = getattr(s, "contraction", None)
        if Cm is not None:
            # CSR of the contraction by orbital: the nonzero C[mu][c] of each column c
            Cm = np.asarray(Cm, np.float64)
            cols = [np.nonzero(Cm[:, c])[0] for c in range(Cm.shape[1])]
            keep.update(con_ptr=np.concatenate([[0], np.cumsum([len(x) for x in cols])]).astype(np.int32),
                        con_idx=np.ascontiguousarray(np.concatenate(cols), np.int32),
                        con_coef=np.ascontiguousarray(np.concatenate([Cm[x, c] for c, x in enumerate(cols)]),
                                                      np.float64))
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        d = SystemDesc(
            n_nuc=len(s.Z), R=p(keep["R"]), Z=p(keep["Z"]), n_basis=len(s.zeta),
            center=p(keep["center"]), l=p(keep["l"]), m=p(keep["m"]), radial=p(keep["radial"]),
            zeta=p(keep["zeta"]), lambda_=p(keep["lam"]), n_up=s.n_up, n_dn=s.n_dn,
            j1_form=s.j1_form, j1_b=p(keep["j1_b"]), j2_form=s.j2_form, n_j2=len(s.j2),
            j2=p(keep["j2"]), precision=precision,
            refresh_every=s.refresh_every if refresh_every is None else refresh_every,
            n_jbasis=LJ, unpaired=p(keep["unpaired"]) if (s.n_up > s.n_dn and not pf) or k_pf else None,
            pairing=pf, pf_k=k_pf,
            **({} if not pf else dict(pf_uu=p(keep["pf_uu"]), pf_dd=p(keep["pf_dd"]),
                                      pf_unpaired_dn=p(keep["pf_dn"]) if k_pf else None)),
            **({} if not LJ else dict(jb_center=p(keep["jb_center"]), jb_l=p(keep["jb_l"]), jb_m=p(keep["jb_m"]),
                                      jb_radial=p(keep["jb_radial"]), jb_zeta=p(keep["jb_zeta"]),
                                      j1_inh=p(keep["j1_inh"]), j3=p(keep["j3"]))),
            **({} if Cm is None else dict(n_contracted=Cm.shape[1], con_ptr=p(keep["con_ptr"]),
                                          con_idx=p(keep["con_idx"]), con_coef=p(keep["con_coef"]))))
        h = ctypes.c_void_p()
        _check(lib.qmc_system_create(ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        self.precision = precision
        self.n_elec = s.n_up + s.n_dn
        self.n_up, self.n_dn, self.L = s.n_up, s.n_dn, len(s.lam)
        self.n_nuc = len(s.Z)
        self.n_jas = len(s.Z) + len(s.j2)
        self.LJ = LJ
        self.n_basis = len(s.zeta)
        # contraction coefficients in the order passed (CSR by orbital): entry t is
        # C[con_mu[t], con_orb[t]]
        self.n_con = 0 if Cm is None else int(keep["con_ptr"][-1])
        if Cm is not None:
            self.con_mu = keep["con_idx"].astype(np.int64)
            self.con_orb = np.repeat(np.arange(Cm.shape[1]), np.diff(keep["con_ptr"]))
        self.pairing = pf
        self.npf = s.n_up + s.n_dn + k_pf if pf else 0

    def set_params(self, R=None, zeta=None, lam=None, jas=None, stream=None):
        """Replace parameters from device tensors (None keeps the current value)."""
        c = lambda t: None if t is None else t.detach().contiguous()
        R, zeta, lam, jas = c(R), c(zeta), c(lam), c(jas)
        _check(load().qmc_system_set_params(self.h, _ptr(R), _ptr(zeta), _ptr(lam), _ptr(jas),
                                            _stream(stream)))

    def set_pfaffian(self, pf_uu=None, pf_dd=None, unpaired=None, unpaired_dn=None, stream=None):
        """Replace the Pfaffian's same-spin blocks / unpaired orbitals from device tensors."""
        c = lambda t: None if t is None else t.detach().contiguous()
        a, b, u, v = c(pf_uu), c(pf_dd), c(unpaired), c(unpaired_dn)
        _check(load().qmc_system_set_pfaffian(self.h, _ptr(a), _ptr(b), _ptr(u), _ptr(v), _stream(stream)))

    def set_jastrow_basis(self, j1_inh=None, j3=None, jb_zeta=None, stream=None):
        """Replace Jastrow-basis coefficients / exponents from device tensors."""
        c = lambda t: None if t is None else t.detach().contiguous()
        j1_inh, j3, jb_zeta = c(j1_inh), c(j3), c(jb_zeta)
        _check(load().qmc_system_set_jastrow_basis(self.h, _ptr(j1_inh), _ptr(j3), _ptr(jb_zeta), _stream(stream)))

    def close(self):
        if getattr(self, "h", None):
            _check(load().qmc_system_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_size(system: JAGPSystem, n_walkers: int, adjoint: bool = True) -> int:
    """Bytes of device memory a walker set occupies (qmc_workspace_size)."""
    n = ctypes.c_size_t()
    _check(load().qmc_workspace_size(system.h, n_walkers, WALKERS_ADJOINT if adjoint else 0, ctypes.byref(n)))
    return n.value


class Walkers:
    """Device state of n_walkers walkers of a JAGPSystem.  adjoint reserves the
    reverse-pass workspace (needed by forces()); workspace: an optional
    caller-owned uint8/float64 device tensor of at least workspace_size bytes
    that the walker set lives in (kept referenced here)."""

    def __init__(self, system: JAGPSystem, n_walkers: int, adjoint: bool = True,
                 workspace: Optional[torch.Tensor] = None):
        self.sys = system
        self.n = n_walkers
        self.adjoint = adjoint
        self.workspace = workspace
        h = ctypes.c_void_p()
        flags = WALKERS_ADJOINT if adjoint else 0
        if workspace is None:
            _check(load().qmc_walkers_create(system.h, n_walkers, flags, None, 0, ctypes.byref(h)))
        else:
            nb = workspace.numel() * workspace.element_size()
            _check(load().qmc_walkers_create(system.h, n_walkers, flags, _ptr(workspace), nb, ctypes.byref(h)))
        self.h = h

    def set_drift_tol(self, tol: float):
        """Residual tolerance of the refresh drift check (status 3); < 0 turns it off."""
        _check(load().qmc_walkers_set_drift_tol(self.h, tol))

    def close(self):
        if getattr(self, "h", None):
            _check(load().qmc_walkers_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def eval_batch(self, r: Optional[torch.Tensor], drift=True, stream=None) -> Dict[str, torch.Tensor]:
        """Evaluate at positions r, or (r None) at the walkers' current positions."""
        dev = r.device if r is not None else torch.device("cuda")
        Wk, N = self.n, self.sys.n_elec
        assert r is None or (r.shape == (Wk, N, 3) and r.dtype == torch.float64)
        f = lambda *sh: torch.empty(*sh, dtype=torch.float64, device=dev)
        out = dict(logabs=f(Wk), sign=f(Wk), drift=f(Wk, N, 3) if drift else None,
                   e_kin=f(Wk), e_loc=f(Wk), status=torch.empty(Wk, dtype=torch.int32, device=dev))
        _check(load().qmc_eval_batch(self.sys.h, self.h, _ptr(r), _ptr(out["logabs"]), _ptr(out["sign"]),
                                     _ptr(out["drift"]), _ptr(out["e_kin"]), _ptr(out["e_loc"]),
                                     _ptr(out["status"]), _stream(stream)))
        return out

    def propose(self, e: int, r_new: torch.Tensor, drift=False, stream=None):
        ratio = torch.empty(self.n, dtype=torch.float64, device=r_new.device)
        dn = torch.empty(self.n, 3, dtype=torch.float64, device=r_new.device) if drift else None
        _check(load().qmc_propose_move(self.sys.h, self.h, e, _ptr(r_new), _ptr(ratio), _ptr(dn),
                                       _stream(stream)))
        return (ratio, dn) if drift else ratio

    def accept(self, e: int, accept: torch.Tensor, status: Optional[torch.Tensor] = None, stream=None):
        assert accept.dtype == torch.uint8
        _check(load().qmc_accept_move(self.sys.h, self.h, e, _ptr(accept), _ptr(status), _stream(stream)))

    def vmc_steps(self, e_start: int, disp: torch.Tensor, unif: torch.Tensor,
                  accept_count: Optional[torch.Tensor] = None, stream=None):
        n_steps = disp.shape[0]
        assert disp.shape == (n_steps, self.n, 3) and unif.shape == (n_steps, self.n)
        _check(load().qmc_vmc_steps(self.sys.h, self.h, e_start, n_steps, _ptr(disp), _ptr(unif),
                                    _ptr(accept_count), _stream(stream)))

    def read(self, item: int, stream=None) -> torch.Tensor:
        Wk, N, nu, nd, L = self.n, self.sys.n_elec, self.sys.n_up, self.sys.n_dn, self.sys.L
        n = self.sys.npf if self.sys.pairing else nu   # G~ (Pfaffian) or W
        shape = {STATE_R: (Wk, N, 3), STATE_LOGABS: (Wk,), STATE_SIGN: (Wk,), STATE_W: (Wk, n, n),
                 STATE_AINV: (Wk, n, n), STATE_PHI: (Wk, N, L), STATE_RESIDUAL: (Wk,), STATE_KEPT: (Wk,)}[item]
        dst = torch.empty(shape, dtype=torch.float64, device="cuda")
        _check(load().qmc_walkers_read(self.h, item, _ptr(dst), _stream(stream)))
        return dst

    def set_timing(self, enable: bool, timers=None):
        """Turn the kernel timers on (all, or only the named ones) or off."""
        if not enable:
            _check(load().qmc_walkers_set_timing(self.h, 0))
        elif timers is None:
            _check(load().qmc_walkers_set_timing(self.h, 1))
        else:
            mask = 0
            for name in timers:
                mask |= 1 << TIMER_NAMES.index(name)
            _check(load().qmc_walkers_set_timing_mask(self.h, mask))

    def timing(self):
        """{timer name: (total ms, launches)}; waits for the recorded events."""
        ms = (ctypes.c_double * len(TIMER_NAMES))()
        n = (ctypes.c_int64 * len(TIMER_NAMES))()
        _check(load().qmc_walkers_timing(self.h, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(TIMER_NAMES)}

    def forces(self, r: torch.Tensor, gbar_logpsi: Optional[torch.Tensor], gbar_eloc: Optional[torch.Tensor],
               per_walker: bool = False, stream=None) -> Dict[str, torch.Tensor]:
        """Gradients of sum_w (gbar_logpsi[w] log|Psi_w| + gbar_eloc[w] e_L,w) (per_walker=False)
        or of each walker's term separately (per_walker=True)."""
        S = self.sys
        Wk, N, A, L, nj = self.n, S.n_elec, S.n_nuc, S.L, S.n_jas
        f = lambda *sh: torch.empty(*sh, dtype=torch.float64, device=r.device)
        if per_walker:
            out = dict(R=f(Wk, A, 3), zeta=f(Wk, S.n_basis), lam=f(Wk, L, L), jas=f(Wk, nj), r=f(Wk, N, 3))
        else:
            out = dict(R=f(A, 3), zeta=f(S.n_basis), lam=f(L, L), jas=f(nj), r=f(Wk, N, 3))
        if S.pairing:       # "lam" is A^{ud}; the skew blocks and both spins' unpaired orbitals
            pre = (Wk,) if per_walker else ()
            out.update(pf_uu=f(*pre, L, L), pf_dd=f(*pre, L, L))
            k = S.npf - S.n_elec
            if k:
                out.update(unpaired=f(*pre, L, k), unpaired_dn=f(*pre, L, k))
        elif S.n_up > S.n_dn:   # unpaired orbitals U [L][k]
            k = S.n_up - S.n_dn
            out["unpaired"] = f(Wk, L, k) if per_walker else f(L, k)
        if S.n_con:             # contraction coefficients, in the CSR order passed
            out["con_coef"] = f(Wk, S.n_con) if per_walker else f(S.n_con)
        LJ = S.LJ
        if LJ:
            pre = (Wk,) if per_walker else ()
            out.update(j1_inh=f(*pre, 2, LJ), j3=f(*pre, 3, LJ, LJ), jb_zeta=f(*pre, LJ))
        g = Grads(dR=_ptr(out["R"]), dzeta=_ptr(out["zeta"]), dlambda=_ptr(out.get("lam")),
                  djas=_ptr(out["jas"]), dr=_ptr(out["r"]), dj1_inh=_ptr(out.get("j1_inh")),
                  dj3=_ptr(out.get("j3")), djb_zeta=_ptr(out.get("jb_zeta")),
                  dunpaired=_ptr(out.get("unpaired")), dcon_coef=_ptr(out.get("con_coef")),
                  dpf_uu=_ptr(out.get("pf_uu")), dpf_dd=_ptr(out.get("pf_dd")),
                  dunpaired_dn=_ptr(out.get("unpaired_dn")))
        _check(load().qmc_forces(S.h, self.h, _ptr(r), 1 if per_walker else 0, _ptr(gbar_logpsi),
                                 _ptr(gbar_eloc), ctypes.byref(g), _stream(stream)))
        return out

    def jastrow_basis_logderiv(self, stream=None):
        """d log Psi / d (j1_inh [Wk, 2, LJ], j3 [Wk, 3, LJ, LJ]) at the current positions."""
        LJ = self.sys.LJ
        f = lambda *sh: torch.empty(*sh, dtype=torch.float64, device="cuda")
        dm, dM = f(self.n, 2, LJ), f(self.n, 3, LJ, LJ)
        _check(load().qmc_jastrow_basis_logderiv(self.sys.h, self.h, _ptr(dm), _ptr(dM), _stream(stream)))
        return dm, dM

    def pfaffian_logderiv(self, stream=None):
        """d log Psi / d (pf_uu, pf_dd, lambda [Wk, L, L] each; unpaired, unpaired_dn [Wk, L, k])."""
        S = self.sys
        k = S.npf - S.n_elec
        f = lambda *sh: torch.empty(*sh, dtype=torch.float64, device="cuda")
        out = dict(uu=f(self.n, S.L, S.L), dd=f(self.n, S.L, S.L), ud=f(self.n, S.L, S.L))
        out.update(unpaired_up=f(self.n, S.L, k) if k else None, unpaired_dn=f(self.n, S.L, k) if k else None)
        _check(load().qmc_pfaffian_logderiv(S.h, self.h, _ptr(out["uu"]), _ptr(out["dd"]), _ptr(out["ud"]),
                                            _ptr(out["unpaired_up"]), _ptr(out["unpaired_dn"]), _stream(stream)))
        return out

    def lrdmc_hops(self, a: float, a_valence: float = 0.0, tf_scale: float = 1.0, gamma: float = 0.0,
                   ratios: bool = True, stream=None) -> Dict[str, torch.Tensor]:
        """Lattice hop ratios [Wk, N, 6] (if requested) and the per-walker terms,
        as a dict keyed by LR_TERMS plus 'ratios' and 'terms' [Wk, 7]."""
        Wk, N = self.n, self.sys.n_elec
        f = lambda *sh: torch.empty(*sh, dtype=torch.float64, device="cuda")
        rt = f(Wk, N, 6) if ratios else None
        terms = f(Wk, len(LR_TERMS))
        prm = LrdmcParams(a=a, a_valence=a_valence, tf_scale=tf_scale, gamma=gamma)
        _check(load().qmc_lrdmc_hops(self.sys.h, self.h, ctypes.byref(prm), _ptr(rt), _ptr(terms),
                                     _stream(stream)))
        out = {k: terms[:, i] for i, k in enumerate(LR_TERMS)}
        out["terms"] = terms
        out["ratios"] = rt
        return out

    def lrdmc_advance(self, xi: torch.Tensor, weight: torch.Tensor, tau_left: torch.Tensor, stream=None):
        """Continuous-time lattice step; weight and tau_left are updated in
        place.  Returns (r_next [Wk, N, 3], hop [Wk])."""
        Wk, N = self.n, self.sys.n_elec
        assert xi.shape == (Wk, 2) and weight.shape == (Wk,) and tau_left.shape == (Wk,)
        r_next = torch.empty(Wk, N, 3, dtype=torch.float64, device="cuda")
        hop = torch.empty(Wk, dtype=torch.int32, device="cuda")
        _check(load().qmc_lrdmc_advance(self.sys.h, self.h, _ptr(xi), _ptr(weight), _ptr(tau_left),
                                        _ptr(r_next), _ptr(hop), _stream(stream)))
        return r_next, hop


def swct(system: JAGPSystem, r: torch.Tensor, dR: torch.Tensor, dr: torch.Tensor, jacobian: bool = False,
         stream=None) -> torch.Tensor:
    """Space-warp total derivatives [Wk, A, 3] from the per-walker partials
    dR [Wk, A, 3] and dr [Wk, N, 3] at the positions r [Wk, N, 3]."""
    Wk = r.shape[0]
    A, N = system.n_nuc, system.n_elec
    assert r.shape == (Wk, N, 3) and dR.shape == (Wk, A, 3) and dr.shape == (Wk, N, 3)
    out = torch.empty(Wk, A, 3, dtype=torch.float64, device=r.device)
    _check(load().qmc_swct(system.h, Wk, _ptr(r), _ptr(dR.contiguous()), _ptr(dr.contiguous()),
                           1 if jacobian else 0, _ptr(out), _stream(stream)))
    return out


def reweight(walkers: Walkers, theta: float, eps: float, stream=None):
    """Reweighting factor R [Wk] and weight [Wk] of the last evaluation."""
    R = torch.empty(walkers.n, dtype=torch.float64, device="cuda")
    w = torch.empty(walkers.n, dtype=torch.float64, device="cuda")
    _check(load().qmc_reweight(walkers.sys.h, walkers.h, theta, eps, _ptr(R), _ptr(w), _stream(stream)))
    return R, w


def sr_step(O: torch.Tensor, e_loc: torch.Tensor, eps: float, weights: Optional[torch.Tensor] = None,
            max_iter: int = 200, tol: float = 1e-12, work: Optional[torch.Tensor] = None, stream=None):
    """Stochastic-reconfiguration step on the device: (delta [P], f [P],
    relative residual [1]) from O [M, P] and e_loc [M]."""
    M, P = O.shape
    assert e_loc.shape == (M,) and (weights is None or weights.shape == (M,))
    lib = load()
    nb = lib.qmc_sr_workspace_size(M, P)
    if work is None or work.numel() * work.element_size() < nb:
        work = torch.empty((nb + 7) // 8, dtype=torch.float64, device=O.device)
    delta = torch.empty(P, dtype=torch.float64, device=O.device)
    f = torch.empty(P, dtype=torch.float64, device=O.device)
    res = torch.empty(1, dtype=torch.float64, device=O.device)
    _check(lib.qmc_sr_step(M, P, _ptr(O.contiguous()), _ptr(e_loc.contiguous()),
                           _ptr(None if weights is None else weights.contiguous()), eps, max_iter, tol,
                           _ptr(delta), _ptr(f), _ptr(res), _ptr(work), work.numel() * work.element_size(),
                           _stream(stream)))
    return delta, f, res


class JAGPFunction(torch.autograd.Function):
    """(log|Psi|, E_loc) of every walker as a differentiable function of the
    electron positions r [Wk,N,3], nuclear positions R [A,3], exponents zeta [L],
    pairing matrix Lambda [L,L] and Jastrow vector [A + n_j2].  The backward
    pass is the library's hand-written adjoint (qmc_forces, summed over walkers).
    Call as JAGPFunction.apply(walkers, r, R, zeta, Lambda, jas)."""

    @staticmethod
    def forward(ctx, walkers, r, R, zeta, lam, jas):
        walkers.sys.set_params(R, zeta, lam, jas)
        out = walkers.eval_batch(r.detach().contiguous(), drift=False)
        ctx.walkers = walkers
        ctx.save_for_backward(r.detach(), R.detach(), zeta.detach(), lam.detach(), jas.detach())
        return out["logabs"], out["e_loc"]

    @staticmethod
    def backward(ctx, g_logabs, g_eloc):
        r, R, zeta, lam, jas = ctx.saved_tensors
        wk = ctx.walkers
        wk.sys.set_params(R, zeta, lam, jas)
        gl = None if g_logabs is None else g_logabs.contiguous()
        ge = None if g_eloc is None else g_eloc.contiguous()
        g = wk.forces(r.contiguous(), gl, ge)
        return None, g["r"], g["R"], g["zeta"], g["lam"], g["jas"]


def philox_draws(seed: int, member: int, n_walkers: int, step: int, sigma: float, stream=None):
    """Device Philox4x32-10 draws of one step: (disp [Wk,3], unif [Wk])."""
    disp = torch.empty(n_walkers, 3, dtype=torch.float64, device="cuda")
    unif = torch.empty(n_walkers, dtype=torch.float64, device="cuda")
    _check(load().qmc_philox_draws(seed, member, n_walkers, step, sigma, _ptr(disp), _ptr(unif), _stream(stream)))
    return disp, unif


class MultiSystem:
    """Several (JAGPSystem, Walkers) pairs moved together by persistent launches."""

    def __init__(self, walkers_list):
        self.members = list(walkers_list)
        n = len(self.members)
        sh = (ctypes.c_void_p * n)(*[w.sys.h for w in self.members])
        wh = (ctypes.c_void_p * n)(*[w.h for w in self.members])
        h = ctypes.c_void_p()
        _check(load().qmc_multi_create(n, sh, wh, ctypes.byref(h)))
        self.h = h

    def autotune(self, stream=None):
        r = ctypes.c_int32()
        g = ctypes.c_int32()
        _check(load().qmc_multi_autotune(self.h, ctypes.byref(r), ctypes.byref(g), _stream(stream)))
        return r.value, g.value

    def vmc_steps(self, n_steps: int, disp=None, unif=None, seed: int = 0, sigma: float = 0.3,
                  use_graph: bool = False, stream=None):
        n = len(self.members)
        if disp is not None:
            dp = (ctypes.c_void_p * n)(*[_ptr(d).value for d in disp])
            up = (ctypes.c_void_p * n)(*[_ptr(u).value for u in unif])
        else:
            dp = up = None
        _check(load().qmc_multi_vmc_steps(self.h, n_steps, dp, up, seed, sigma, 1 if use_graph else 0,
                                          _stream(stream)))

    def close(self):
        if getattr(self, "h", None):
            _check(load().qmc_multi_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
