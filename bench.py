"""Benchmark of the batched JAGP hot path on one MI355X.

One step = one from-scratch evaluation of every walker (basis -> P = Phi Lambda
-> W -> FP64 LU/inverse -> cofactor products -> local energy) followed by one
sweep of single-electron Metropolis moves (every electron once, device-side
accept, FP64 delayed low-rank updates of W^{-1}, FP64 refresh after 32 moves of
one spin and at each change of spin).
Workload: 40 nuclei, 160 electrons (80/80), 600 Gaussian basis functions,
1024 walkers (synthetic, seeded).

Prints ONE JSON line.  `value` is walker-electron moves/s over the move
sweeps of the timed steps; E_loc evaluations/s over their evaluations are
reported beside it, with the error against the CPU oracle on sampled walkers,
the roofline of the dominant kernel and the oracle's own CPU throughput.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

METRIC = "walker-electron moves/s + E_loc evals/s at 160e, mixed vs FP64, err vs oracle"
HBM_PEAK_GBS = 8000.0
INT8_PEAK_TOPS = 5000.0
# the evaluation's P = Phi Lambda product: FP64 MFMA (fp64), FP32 MFMA (fp32),
# int8 MFMA digit products (mixed, mixed_fp32_rows, bf16: refined evaluations)
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "mixed": INT8_PEAK_TOPS, "mixed_fp32_rows": INT8_PEAK_TOPS,
                    "bf16": INT8_PEAK_TOPS}
OZ_DIGITS = 7          # int8 digits per FP64 row in the refined products
PRECISIONS = ("fp64", "mixed", "mixed_fp32_rows", "bf16", "fp32")
# accuracy bar of each mode's ratios and evaluations against the oracle
BARS = {"fp64": 1e-10, "mixed": 1e-6, "mixed_fp32_rows": 1e-6, "bf16": 1e-6, "fp32": 1e-6}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--walkers", type=int, default=1024)
    ap.add_argument("--precision", default="fp64", choices=list(PRECISIONS),
                    help="fp64 (QMC_FP64); mixed (QMC_REFINED: int8-refined products, screened FP64 "
                         "proposals); mixed_fp32_rows (QMC_MIXED: refined evaluations, FP32 move rows); "
                         "bf16 (QMC_MIXED_BF16: BF16 move rows); fp32 (QMC_W_FP32: FP32 products and rows)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-walkers", type=int, default=4)
    ap.add_argument("--only", action="store_true", help="run the headline precision only")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


# Sources of the move kernels: a recorded counter measurement is reported only
# while these files are unchanged.
ROWS_SOURCES = ("paper_2002_07401_amd/csrc/move.hip", "paper_2002_07401_amd/csrc/move_dev.h",
                "paper_2002_07401_amd/csrc/move_staged.h", "paper_2002_07401_amd/csrc/sweep.hip",
                "paper_2002_07401_amd/csrc/internal.h")


def rows_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ROWS_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(tag, precision, walkers):
    """HBM bytes per launch of a move kernel (tag: sweep, propose_rows,
    propose_screened or accept_prep) from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes, each scaled by the same counter over a
    plain copy of known size), or None when the summary is missing, was taken
    on another configuration, or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"{tag}_mol160e_{precision}_pmc.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    if rec.get("source_sha256") != rows_source_hash() or rec.get("walkers") != str(walkers):
        return None
    try:
        return int(float(rec["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def copy_probe(mib):
    """A plain elementwise copy (read mib MiB, write mib MiB) for calibrating
    the FETCH_SIZE / WRITE_SIZE counters."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(2):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst


def kernel_models(s, Wk, esz, acc_rate, kept=None, p_rows=None):
    """Algorithmic bytes / flops per launch of the main kernels.

    propose (the streaming kernel): every walker reads the N_other x L rows of P
             of the opposite spin (esz bytes each), psi(r') (8 L), the current
             W^{-1} column / row of the moved electron (8 N_other, assembled by the
             set-up kernel), and writes the new W row (8 N_other).  Screened
             proposals (kept = average number of basis functions streamed):
             kept columns of N_other FP64 values, the kept functions' indices and
             values (12 kept), the inverse column (8 N_other) and the new row
             (8 N_other).
    accept:  the Metropolis accept fused with the next proposal's set-up (the
             kernel of 150 of the 160 steps of a sweep), per walker with m
             buffered moves: reads the m rows of V and D and S^{-1}
             (8 (2 m n + m^2)), the new and old W line, v0 and the next
             electron's A0 line (32 n), z (8 m) and the positions (24 N); an
             accepted walker also reads psi(r') (8 L) and writes d and v
             (16 n), the bordered S^{-1} (8 (m+1)^2), the W line (8 n) and the
             basis row (esz L); every walker writes psi(r') of the next
             electron (8 Lp), v0 and the inverse line (16 n) and t, z
             (16 m); screened proposals add the column maxima (8 L) and the
             kept list (12 kept).  m is averaged over a sweep: the buffer
             restarts at every refresh (after min(refresh_every, 64) moves of
             one spin and at each change of spin) and grows by the
             acceptance rate per move.
    P_build: the evaluation's P = Phi Lambda, 2 L^2 flops per basis row over
             Wk * p_rows rows: p_rows = N when both spins are built; after a
             sweep the up rows are current and only the rows of the down
             electrons that moved are built (n_dn times the share that moved;
             the one-spin rebuilds before moves have a timer of their own).
    """
    L, N, n = s.n_basis, s.n_up + s.n_dn, s.n_up
    cap = min(s.refresh_every, 64)
    cycles = [cap] * (n // cap) + ([n % cap] if n % cap else [])
    m = acc_rate * sum(c * (c - 1) / 2 for c in cycles) / n
    if kept is None:
        prop = Wk * (esz * n * L + 8 * L + 8 * n + 8 * n)
    else:
        prop = Wk * (kept * (8 * n + 12) + 16 * n)
    Lp = (L + 31) // 32 * 32
    acc = Wk * (8 * (2 * m * n + m * m) + 32 * n + 8 * m + 24 * N
                + acc_rate * (8 * L + 16 * n + 8 * (m + 1) ** 2 + 8 * n + esz * L)
                + 8 * Lp + 16 * n + 16 * m
                + (8 * L + 12 * kept if kept is not None else 0))
    pflops = 2.0 * L * L * Wk * (N if p_rows is None else p_rows)
    return {"propose": ("hbm", prop), "accept": ("hbm", acc), "P_build": ("mfma", pflops)}


def host_cpu():
    """Model name of the host processor and the cores this process may use."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, len(os.sched_getaffinity(0))


def prop_roofline(models, tim):
    """Roofline fields of the proposal stream from the timed steps (None when
    every proposal ran inside the persistent sweep)."""
    ms, cnt = tim["propose"]
    if not cnt:
        return None
    avg = ms / cnt
    ach = models["propose"][1] / (avg * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "avg_launch_us": round(avg * 1e3, 2)}


def sweep_bytes(models, tim, moves):
    """Algorithmic bytes per launch of the persistent sweep over the timed
    steps: every proposal not launched on its own ran inside a sweep, and every
    sweep launch ends with a proposal whose accept is a launch of its own, so a
    sweep of k proposals holds k - 1 fused accepts (each priced as the fused
    accept kernel: propose and accept bytes per walker from kernel_models)."""
    launches = tim["sweep"][1]
    if not launches:
        return None
    props = moves - tim["propose"][1]
    accs = props - launches
    return (props * models["propose"][1] + accs * models["accept"][1]) / launches


def cpu_baseline(w, n_walk=8, n_moves=320, n_eval=32, n_moves_1t=40):
    """The CPU oracle, untuned, on a bounded sample of the same workload: with
    torch's default thread count, and on one thread for a shorter chain."""
    from oracle import jagp as O
    from workloads import configs as C
    sy = O.from_workload_system(w.system)
    t0 = time.perf_counter()
    O.evaluate(sy, torch.tensor(w.r0[:n_eval]))
    t_eval = time.perf_counter() - t0
    r = torch.tensor(w.r0[:n_walk])
    disp, unif = C.chain_arrays(77, n_moves, n_walk)
    t0 = time.perf_counter()
    O.run_chain(sy, r, torch.tensor(disp), torch.tensor(unif))
    t_moves = time.perf_counter() - t0
    threads = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        O.run_chain(sy, r, torch.tensor(disp[:n_moves_1t]), torch.tensor(unif[:n_moves_1t]))
        t_1t = time.perf_counter() - t0
    finally:
        torch.set_num_threads(threads)
    model, avail = host_cpu()
    return {
        "value": n_walk * n_moves / t_moves, "unit": "walker-electron moves/s",
        "cores": threads, "kind": "oracle",
        "sample": f"{n_walk} walkers x {n_moves} single-electron moves (each move re-evaluates Psi "
                  f"from scratch) and E_loc evaluations of {n_eval} walkers, same workload",
        "eloc_evals_per_s": n_eval / t_eval,
        "one_thread": {"value": n_walk * n_moves_1t / t_1t, "unit": "walker-electron moves/s",
                       "sample": f"{n_walk} walkers x {n_moves_1t} moves"},
        "host_cpu": model, "host_cores_available": avail,
        "seconds": round(t_eval + t_moves + t_1t, 2),
    }


def run_precision(P, C, w, args, precision):
    """Timed steps at one precision; returns the measurement record."""
    from oracle import jagp as O
    dev = torch.device("cuda:0")
    s = w.system
    N = s.n_up + s.n_dn
    Wk = args.walkers
    prec = {"fp64": P.QMC_FP64, "mixed": P.QMC_REFINED, "mixed_fp32_rows": P.QMC_MIXED, "bf16": P.QMC_MIXED_BF16,
            "fp32": P.QMC_W_FP32}[precision]
    esz = {"fp64": 8, "mixed": 8, "bf16": 2}.get(precision, 4)
    screened = precision == "mixed"
    sysh = P.JAGPSystem(s, precision=prec)
    wk = P.Walkers(sysh, Wk, adjoint=False)
    n_tot = args.warmup + args.steps
    # one more step after the timed ones: the per-kernel breakdown
    disp, unif = C.chain_arrays(20020740, (n_tot + 1) * N, Wk)
    disp = torch.tensor(disp, device=dev).view(n_tot + 1, N, Wk, 3)
    unif = torch.tensor(unif, device=dev).view(n_tot + 1, N, Wk)
    cnt = torch.zeros(Wk, dtype=torch.int32, device=dev)
    wk.eval_batch(torch.tensor(w.r0, device=dev), drift=True)   # the starting positions

    def step(k, ev=None):
        # E_loc at the chain's current positions, then one sweep of moves
        if ev: ev[0].record()
        wk.eval_batch(None, drift=True)
        if ev: ev[1].record()
        wk.vmc_steps(0, disp[k], unif[k], cnt)
        if ev: ev[2].record()

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    cnt.zero_()
    # the timed steps record events only around the kernels a roofline is
    # reported for (every timed launch adds two event records to the stream)
    wk.set_timing(True, timers=("sweep", "propose", "accept", "P_build"))
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k, evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tim = wk.timing()
    n_acc = cnt.sum().item()
    wk.set_timing(True)
    r_a = wk.read(P.STATE_R)
    step(n_tot)
    one = wk.timing()
    wk.set_timing(False)
    # the share of each spin's electrons that moved in a sweep (measured on
    # this step): FP64, FP32 and the refined mode build only those P rows
    moved = (wk.read(P.STATE_R) != r_a).any(-1)
    f_up = moved[:, :s.n_up].double().mean().item()
    f_dn = moved[:, s.n_up:].double().mean().item()
    t_eval = sum(e[0].elapsed_time(e[1]) for e in evs) / 1e3
    t_move = sum(e[1].elapsed_time(e[2]) for e in evs) / 1e3
    moves = args.steps * N * Wk
    acc_rate = n_acc / moves

    # screened proposals: basis functions streamed per proposal over one sweep
    r_cur = wk.read(P.STATE_R)
    kept = None
    if screened:
        ks = []
        for t in range(N):
            wk.vmc_steps(t, disp[0][t:t + 1].contiguous(), unif[0][t:t + 1].contiguous())
            ks.append(wk.read(P.STATE_KEPT))
        kept = torch.stack(ks).mean().item()
        r_cur = wk.read(P.STATE_R)

    # error against the CPU oracle on sampled walkers at the final positions: an
    # evaluation (log|Psi|, E_loc) and the ratios of proposals of two up and two
    # down electrons (the definition: two full evaluations)
    idx = np.linspace(0, Wk - 1, args.oracle_walkers).round().astype(int).tolist()
    err = {}
    if idx:
        out = wk.eval_batch(r_cur, drift=True)
        torch.cuda.synchronize()
        sy = O.from_workload_system(s)
        rc = r_cur.cpu()
        ref = O.evaluate(sy, rc[idx])
        for key in ("logabs", "e_loc"):
            d = (out[key].cpu()[idx] - ref[key]).abs() / ref[key].abs().clamp(min=1.0)
            err[key] = float(f"{float(d.max()):.3e}")
        g = torch.Generator().manual_seed(5)
        rmax = 0.0
        for e in (3, s.n_up - 1, s.n_up, N - 7):
            rn = rc[:, e] + 0.3 * torch.randn(Wk, 3, generator=g, dtype=torch.float64)
            wk.eval_batch(r_cur, drift=False)
            ratio = wk.propose(e, rn.to(dev).contiguous()).cpu()[idx]
            rr = O.move_ratio(sy, rc[idx], e, rn[idx])
            rmax = max(rmax, float(((ratio - rr).abs() / rr.abs().clamp(min=1.0)).max()))
        err["ratio"] = float(f"{rmax:.3e}")
        err["bar"] = BARS[precision]
        err["conforming"] = bool(max(err["logabs"], err["e_loc"], err["ratio"]) <= BARS[precision])

    # roofline of the dominant kernel among those with a model (proposal
    # stream, fused accept, P product: largest summed time in the timed
    # steps); the kernel with the largest summed time overall is named beside it
    # the timed evaluations run at the chain's positions after full sweeps: in
    # FP64, FP32 and the refined mode the up rows of P are current from the
    # rebuild between the halves of the sweep, and their P_build builds the
    # rows of the down electrons that moved in the sweep (the rebuild, those of
    # the up electrons); the other modes rebuild their FP64 P for both spins
    part = precision in ("fp64", "fp32", "mixed")
    p_rows = s.n_dn * f_dn if part else N
    rb_rows = s.n_up * f_up if part else s.n_up
    models = kernel_models(s, Wk, esz, acc_rate, kept, p_rows)
    sw = sweep_bytes(models, tim, args.steps * N)
    if sw is not None:
        models["sweep"] = ("hbm", sw)
    dominant = max(one, key=lambda k: one[k][0])
    dom = max((k for k in models if tim.get(k, (0.0, 0))[1]), key=lambda k: tim[k][0])
    bound, units = models[dom]
    avg_ms = tim[dom][0] / max(tim[dom][1], 1)
    if bound == "hbm":
        achieved = units / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": recorded_traffic({"propose": "propose_screened" if screened else "propose_rows",
                                             "accept": "accept_prep", "sweep": "sweep"}[dom], precision, Wk),
                "bytes_per_launch": int(units), "avg_launch_us": round(avg_ms * 1e3, 2)}
    else:
        peak = MFMA_PEAK_TFLOPS[precision]
        achieved = units / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 2), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                "flops_per_launch": int(units), "avg_launch_us": round(avg_ms * 1e3, 2)}
    steps = step_rooflines(s, Wk, precision, one, roof if roof["kernel"] == "propose" else
                           prop_roofline(models, tim), models["accept"][1], p_rows,
                           roof if roof["kernel"] == "sweep" else None, rb_rows)
    # MFMA use of the geminal build's dominant product (P = Phi Lambda in the
    # evaluations of the timed steps).  Refined modes: int8 operations of the
    # digit products (the P_build timer also covers the digit split) against
    # the int8 peak, and the FP64-equivalent rate beside it
    pf_ms = tim["P_build"][0] / max(tim["P_build"][1], 1)
    if not tim["P_build"][1]:
        wmfma = None   # (no evaluation of the timed steps built P)
    elif precision in ("fp64", "fp32"):
        pf_tf = models["P_build"][1] / (pf_ms * 1e-3) / 1e12
        wmfma = {"kernel": "P_build", "instruction": "v_mfma_f64_16x16x4f64" if precision == "fp64"
                 else "v_mfma_f32_16x16x4f32", "achieved": round(pf_tf, 2), "peak": MFMA_PEAK_TFLOPS[precision],
                 "unit": "TFLOP/s", "frac": round(pf_tf / MFMA_PEAK_TFLOPS[precision], 4),
                 "flops_per_launch": int(models["P_build"][1]), "rows_per_walker": round(p_rows, 2),
                 "avg_launch_us": round(pf_ms * 1e3, 2)}
    else:
        Lp = (s.n_basis + 31) // 32 * 32
        ops = 2.0 * Lp * Lp * p_rows * Wk * OZ_DIGITS * (OZ_DIGITS + 1) // 2
        int8 = ops / (pf_ms * 1e-3) / 1e12
        wmfma = {"kernel": "P_build", "instruction": "v_mfma_i32_32x32x32_i8", "achieved": round(int8, 1),
                 "peak": INT8_PEAK_TOPS, "unit": "TOP/s", "frac": round(int8 / INT8_PEAK_TOPS, 4),
                 "ops_per_launch": int(ops), "digit_products": OZ_DIGITS * (OZ_DIGITS + 1) // 2,
                 "fp64_equivalent_TFLOPs": round(models["P_build"][1] / (pf_ms * 1e-3) / 1e12, 2),
                 "rows_per_walker": round(p_rows, 2), "avg_launch_us": round(pf_ms * 1e3, 2)}
    wk.close()
    sysh.close()
    return {
        "mode": {"fp64": "QMC_FP64", "mixed": "QMC_REFINED", "mixed_fp32_rows": "QMC_MIXED",
                 "bf16": "QMC_MIXED_BF16", "fp32": "QMC_W_FP32"}[precision],
        "moves_per_s": round(moves / t_move, 1),
        "eloc_evals_per_s": round(Wk * args.steps / t_eval, 1),
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "acceptance": round(acc_rate, 4),
        "err_vs_oracle": {"walkers": idx, **err},
        "kernel_ms": {k: round(v[0], 3) for k, v in tim.items() if v[1]},
        "kernel_launches": {k: v[1] for k, v in tim.items() if v[1]},
        "kernel_ms_one_step": {k: round(v[0], 3) for k, v in one.items() if v[1]},
        "kernel_launches_one_step": {k: v[1] for k, v in one.items() if v[1]},
        "dominant_kernel": dominant,
        "roofline": roof,
        "w_build_mfma": wmfma,
        "step_rooflines": steps,
        **({"screened_functions_per_proposal": round(kept, 1), "basis_functions": s.n_basis} if screened else {}),
    }


def forces_leg(P, C, reps=5):
    """Adjoint cost on the 80-electron workload: E_loc evaluation vs the full
    reverse pass (gradients of log|Psi| and E_loc w.r.t. R, zeta, Lambda,
    Jastrow and r), 512 walkers, FP64."""
    dev = torch.device("cuda:0")
    w = C.forces_20nuc_80e()
    Wk = w.r0.shape[0]
    sysh = P.JAGPSystem(w.system)
    wk = P.Walkers(sysh, Wk)
    r = torch.tensor(w.r0, device=dev)
    gl = torch.ones(Wk, dtype=torch.float64, device=dev)
    ge = torch.ones(Wk, dtype=torch.float64, device=dev)
    wk.eval_batch(r)
    wk.forces(r, gl, ge)
    torch.cuda.synchronize()
    te, tf = [], []
    for _ in range(reps):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        wk.eval_batch(r)
        e1.record()
        wk.forces(r, gl, ge)
        e2.record()
        torch.cuda.synchronize()
        te.append(e0.elapsed_time(e1))
        tf.append(e1.elapsed_time(e2))
    te, tf = float(np.median(te)), float(np.median(tf))
    wk.close()
    sysh.close()
    return {"workload": "forces_20nuc_80e", "walkers": Wk, "eval_ms": round(te, 3),
            "forces_ms": round(tf, 3), "forces_over_eval": round(tf / te, 2),
            "grad_evals_per_s": round(Wk / (tf * 1e-3), 1),
            "note": "forces_ms includes its own re-evaluation; the paper quotes ~4x for energy+forces"}


def multi_leg(P, C, precision="fp32", replays=3):
    """Eight systems with 16..256 electrons, 256 walkers each (2048 walkers),
    with FP32 rows, BF16 rows or in QMC_REFINED ("mixed": int8-refined
    products, screened FP64 proposals), moved together by the persistent
    multi-system launches: autotuned, one
    graph of 768 steps (the schedule period of all members) replayed.  Beside
    it the same members moved one system at a time with qmc_vmc_steps."""
    dev = torch.device("cuda:0")
    prec = {"fp64": P.QMC_FP64, "fp32": P.QMC_W_FP32, "bf16": P.QMC_MIXED_BF16, "mixed": P.QMC_REFINED}[precision]
    members = []
    for n in C.MULTI_SIZES:
        w = C.multi_system(n)
        sysh = P.JAGPSystem(w.system, precision=prec)
        wk = P.Walkers(sysh, w.r0.shape[0], adjoint=False)
        wk.eval_batch(torch.tensor(w.r0, device=dev))
        members.append((w, sysh, wk))
    m = P.MultiSystem([wk for _, _, wk in members])
    rows, grid = m.autotune()
    period = 768
    m.vmc_steps(period, seed=11, sigma=0.3, use_graph=True)      # capture + first replay
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(replays):
        m.vmc_steps(period, seed=11, sigma=0.3, use_graph=True)
    e1.record()
    torch.cuda.synchronize()
    t_multi = e0.elapsed_time(e1) / 1e3
    n_walk = sum(w.r0.shape[0] for w, _, _ in members)
    moves = replays * period * n_walk
    # one system at a time, same number of steps, host-driven launches
    steps = 96
    draws = [C.chain_arrays(31 + k, steps, w.r0.shape[0]) for k, (w, _, _) in enumerate(members)]
    draws = [(torch.tensor(d, device=dev), torch.tensor(u, device=dev)) for d, u in draws]
    torch.cuda.synchronize()
    e0.record()
    for k, (_, _, wk) in enumerate(members):
        wk.vmc_steps(0, draws[k][0], draws[k][1])
    e1.record()
    torch.cuda.synchronize()
    t_seq = e0.elapsed_time(e1) / 1e3
    m.close()
    return {"workload": "multi_8sys_16to256e", "walkers": n_walk, "precision": precision,
            "moves_per_s": round(moves / t_multi, 1), "graph_steps": period, "replays": replays,
            "autotuned_rows_per_item": rows, "autotuned_grid": grid,
            "one_system_at_a_time_moves_per_s": round(steps * n_walk / t_seq, 1)}


def lrdmc_leg(P, C, iters=10):
    """Lattice-regularised DMC on the 160-electron workload, 1024 walkers,
    FP64, double grid (0.1 / 0.4 bohr hops, fixed-node gamma 0.5): `iters`
    iterations of evaluation -> 6N hop ratios and Green's function terms ->
    continuous-time step.  Error of sampled hop ratios (walker 0, electrons 0
    and 80) against the oracle's full re-evaluations."""
    from oracle import jagp as O
    from oracle import lrdmc as L
    dev = torch.device("cuda:0")
    w = C.mol_40nuc_160e()
    s = w.system
    Wk, N, Lb = w.r0.shape[0], s.n_up + s.n_dn, s.n_basis
    prm = C.LRDMC_DOUBLE
    sysh = P.JAGPSystem(s)
    wk = P.Walkers(sysh, Wk, adjoint=False)
    r0 = torch.tensor(w.r0, device=dev)
    xi = torch.tensor(C.lrdmc_draws(17, iters + 1, Wk), device=dev)
    weight = torch.ones(Wk, dtype=torch.float64, device=dev)
    tau = torch.empty(Wk, dtype=torch.float64, device=dev)
    # warm-up iteration, then the sampled error at the starting positions
    wk.eval_batch(r0)
    g = wk.lrdmc_hops(**prm)
    torch.cuda.synchronize()
    sy = O.from_workload_system(s)
    rc = r0[:1].cpu()
    a_i = L.mesh(sy, rc, prm["a"], prm["a_valence"], prm["tf_scale"])
    err = 0.0
    for e in (0, s.n_up):
        for k, (sg, ax) in enumerate(L.DIRS):
            rn = rc[:, e].clone()
            rn[0, ax] += sg * a_i[0, e]
            ref = O.move_ratio(sy, rc, e, rn)[0]
            err = max(err, float((g["ratios"][0, e, k].cpu() - ref).abs() / max(abs(float(ref)), 1.0)))
    r = r0
    wk.set_timing(True)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(iters)]
    hops = 0
    cnt = torch.zeros((), dtype=torch.int64, device=dev)
    for t in range(iters):
        tau.fill_(C.LRDMC_TAU)
        ev[t][0].record()
        wk.eval_batch(r, drift=False)
        ev[t][1].record()
        wk.lrdmc_hops(**prm, ratios=False)
        ev[t][2].record()
        r, hop = wk.lrdmc_advance(xi[t], weight, tau)
        ev[t][3].record()
        cnt += (hop >= 0).sum()
    torch.cuda.synchronize()
    tim = wk.timing()
    wk.set_timing(False)
    hops = int(cnt.item())
    t_eval = sum(e[0].elapsed_time(e[1]) for e in ev) / 1e3
    t_hops = sum(e[1].elapsed_time(e[2]) for e in ev) / 1e3
    t_adv = sum(e[2].elapsed_time(e[3]) for e in ev) / 1e3
    t_all = sum(e[0].elapsed_time(e[3]) for e in ev) / 1e3
    wk.close()
    sysh.close()
    return {"workload": "mol_40nuc_160e", "walkers": Wk, "precision": "fp64",
            "grid": f"double ({prm['a']} / {prm['a_valence']} bohr)", "gamma": prm["gamma"],
            "iterations": iters, "lrdmc_steps_per_s": round(iters * Wk / t_all, 1),
            "hop_ratios_per_s": round(iters * Wk * 6 * N / t_hops, 1),
            "hop_basis_values_per_s": round(iters * Wk * 6 * N * Lb / t_hops, 1),
            "eval_ms": round(1e3 * t_eval / iters, 3), "hops_ms": round(1e3 * t_hops / iters, 3),
            "advance_ms": round(1e3 * t_adv / iters, 3), "hops_made": hops,
            "kernel_ms": {k: round(tim[k][0] / iters, 3) for k in ("lrdmc_hops", "lrdmc_step")},
            "ratio_err_vs_oracle": float(f"{err:.3e}")}


def large_leg(P, C, steps=128, Wk=256, fw=32, refined=False):
    """The 1024-electron workload (256 nuclei, L = 4096, Lambda banded at 8
    bohr; n = 512 per spin, so the blocked Gauss-Jordan refresh), 256 walkers:
    one evaluation and `steps` Metropolis moves (refresh after 64 moves of one
    spin); error of the evaluation against the oracle on one walker.  FP64:
    forces through the adjoint on fw walkers.  refined: QMC_REFINED (int8
    digit products skipping Lambda's zero tiles, screened proposals), with
    the basis functions streamed per proposal."""
    from oracle import jagp as O
    dev = torch.device("cuda:0")
    w = C.large_256nuc_1024e(n_walkers=Wk)
    sysh = P.JAGPSystem(w.system, precision=P.QMC_REFINED if refined else P.QMC_FP64)
    wk = P.Walkers(sysh, Wk, adjoint=False)
    r = torch.tensor(w.r0, device=dev)
    d, u = C.chain_arrays(41, steps, Wk)
    d, u = torch.tensor(d, device=dev), torch.tensor(u, device=dev)
    cnt = torch.zeros(Wk, dtype=torch.int32, device=dev)
    wk.eval_batch(r)
    torch.cuda.synchronize()
    wk.set_timing(True)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    out = wk.eval_batch(r, drift=True)
    e1.record()
    wk.vmc_steps(0, d, u, cnt)
    e2.record()
    torch.cuda.synchronize()
    tim = wk.timing()
    wk.set_timing(False)
    t_eval, t_move = e0.elapsed_time(e1) / 1e3, e1.elapsed_time(e2) / 1e3
    ref = O.evaluate(O.from_workload_system(w.system), torch.tensor(w.r0[:1]))
    err = {k: float(f"{float(((out[k].cpu()[:1] - ref[k]).abs() / ref[k].abs().clamp(min=1.0)).max()):.3e}")
           for k in ("logabs", "e_loc")}
    rec = {"workload": "large_256nuc_1024e", "walkers": Wk, "precision": "refined" if refined else "fp64",
           "eloc_evals_per_s": round(Wk / t_eval, 1), "moves_per_s": round(steps * Wk / t_move, 1),
           "acceptance": round(cnt.sum().item() / (steps * Wk), 4), "moves": steps,
           "err_vs_oracle": {"walkers": [0], **err},
           "kernel_ms": {k: round(v[0], 3) for k, v in tim.items() if v[1]},
           "kernel_launches": {k: v[1] for k, v in tim.items() if v[1]}}
    if refined:
        rec["screened_functions_per_proposal"] = round(wk.read(P.STATE_KEPT).mean().item(), 1)
        rec["basis_functions"] = w.system.n_basis
        wk.close()
        sysh.close()
        return rec
    wk.close()
    # forces via the adjoint on `fw` walkers (the reverse-pass workspace is
    # some 0.2 GB per walker at this size): one evaluation against one call
    # of qmc_forces (which re-evaluates), walker-summed gradients, median of 3
    wf = P.Walkers(sysh, fw)
    rf = r[:fw].contiguous()
    gl = torch.ones(fw, dtype=torch.float64, device=dev)
    wf.forces(rf, gl, gl)
    torch.cuda.synchronize()
    te, tf = [], []
    for _ in range(3):
        f0, f1, f2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        f0.record()
        wf.eval_batch(rf)
        f1.record()
        wf.forces(rf, gl, gl)
        f2.record()
        torch.cuda.synchronize()
        te.append(f0.elapsed_time(f1))
        tf.append(f1.elapsed_time(f2))
    te, tf = float(np.median(te)), float(np.median(tf))
    wf.close()
    sysh.close()
    rec["forces"] = {"walkers": fw, "eval_ms": round(te, 3), "forces_ms": round(tf, 3),
                     "forces_over_eval": round(tf / te, 2), "grad_evals_per_s": round(fw / (tf * 1e-3), 1)}
    return rec


def pfaffian_leg(P, C, steps=160, Wk=512):
    """The 80-electron Pfaffian (G~ 80 x 80, triplet blocks, L = 300), 512
    walkers, FP64: one evaluation and `steps` Metropolis moves (refresh every
    32 moves); error of the evaluation against the oracle on one walker; the
    adjoint's cost against an evaluation; and QMC_REFINED evaluations (B rows
    from int8 digit products) against the FP64 ones, with their error."""
    from oracle import jagp as O
    dev = torch.device("cuda:0")
    w = C.pfaffian_20nuc_80e(n_walkers=Wk)
    sysh = P.JAGPSystem(w.system)
    wk = P.Walkers(sysh, Wk)
    r = torch.tensor(w.r0, device=dev)
    d, u = C.chain_arrays(43, steps, Wk)
    d, u = torch.tensor(d, device=dev), torch.tensor(u, device=dev)
    cnt = torch.zeros(Wk, dtype=torch.int32, device=dev)
    wk.eval_batch(r)
    wk.vmc_steps(0, d[:8].contiguous(), u[:8].contiguous())   # warm-up
    torch.cuda.synchronize()
    wk.set_timing(True)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    out = wk.eval_batch(r, drift=True)
    e1.record()
    wk.vmc_steps(0, d, u, cnt)
    e2.record()
    torch.cuda.synchronize()
    tim = wk.timing()
    wk.set_timing(False)
    t_eval, t_move = e0.elapsed_time(e1) / 1e3, e1.elapsed_time(e2) / 1e3
    ref = O.evaluate(O.from_workload_system(w.system), torch.tensor(w.r0[:1]))
    err = {k: float(f"{float(((out[k].cpu()[:1] - ref[k]).abs() / ref[k].abs().clamp(min=1.0)).max()):.3e}")
           for k in ("logabs", "e_loc")}
    s = w.system
    n, Lp = s.n_up + s.n_dn, (len(s.lam) + 31) // 32 * 32
    prop = tim["propose"]
    # algorithmic bytes of one proposal launch: the n B rows and the inverse column of every walker
    prop_bytes = Wk * (n * Lp * 8 + n * 8)
    prop_us = 1e3 * prop[0] / max(prop[1], 1)
    # adjoint (log|Psi| and e_L weights, summed over walkers) against one evaluation
    one = torch.ones(Wk, dtype=torch.float64, device=dev)
    rf = wk.read(P.STATE_R)
    wk.forces(rf, one, one)
    torch.cuda.synchronize()
    f0, f1, f2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    reps = 3
    f0.record()
    for _ in range(reps):
        wk.eval_batch(rf)
    f1.record()
    for _ in range(reps):
        wk.forces(rf, one, one)
    f2.record()
    torch.cuda.synchronize()
    t_ev, t_fo = f0.elapsed_time(f1) / reps, f1.elapsed_time(f2) / reps
    wk.set_timing(True)
    wk.eval_batch(rf)
    torch.cuda.synchronize()
    b_fp64 = wk.timing()["P_build"][0]
    wk.set_timing(False)
    # QMC_REFINED: the B rows of the evaluation from the int8 digit products
    # (G~, Pf, the inverse and the moves FP64), at the chain's final positions
    sr = P.JAGPSystem(w.system, precision=P.QMC_REFINED)
    wr = P.Walkers(sr, Wk, adjoint=False)
    wr.eval_batch(rf)
    torch.cuda.synchronize()
    g0, g1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
    g0.record()
    for _ in range(reps):
        outr = wr.eval_batch(rf)
    g1.record()
    torch.cuda.synchronize()
    t_evr = g0.elapsed_time(g1) / reps
    wr.set_timing(True)
    wr.eval_batch(rf)
    torch.cuda.synchronize()
    b_ref = wr.timing()["P_build"][0]
    wr.close()
    sr.close()
    refr = O.evaluate(O.from_workload_system(w.system), rf[:1].cpu())
    errr = {k: float(f"{float(((outr[k].cpu()[:1] - refr[k]).abs() / refr[k].abs().clamp(min=1.0)).max()):.3e}")
            for k in ("logabs", "e_loc")}
    refined = {"mode": "QMC_REFINED", "eval_ms": round(t_evr, 3), "eval_over_fp64": round(t_ev / t_evr, 3),
               "B_rows_ms": round(b_ref, 3), "B_rows_fp64_ms": round(b_fp64, 3),
               "err_vs_oracle": {"walkers": [0], **errr}}
    wk.close()
    sysh.close()
    return {"workload": "pfaffian_20nuc_80e", "walkers": Wk, "precision": "fp64", "pfaffian_dim": n,
            "refined": refined,
            "forces_ms": round(t_fo, 3), "eval_ms": round(t_ev, 3), "forces_over_eval": round(t_fo / t_ev, 2),
            "eloc_evals_per_s": round(Wk / t_eval, 1), "moves_per_s": round(steps * Wk / t_move, 1),
            "acceptance": round(cnt.sum().item() / (steps * Wk), 4), "moves": steps,
            "propose_avg_us": round(prop_us, 2),
            "propose_GBps": round(prop_bytes / (prop_us * 1e-6) / 1e9, 1),
            "err_vs_oracle": {"walkers": [0], **err},
            "kernel_ms": {k: round(v[0], 3) for k, v in tim.items() if v[1]},
            "kernel_launches": {k: v[1] for k, v in tim.items() if v[1]}}


def sr_leg(P, M=4096, Pn=8192, iters=40, eps=1e-3):
    """Stochastic-reconfiguration step on the device: M samples x Pn
    parameters of synthetic logarithmic derivatives (correlated Gaussian
    columns with scales spread over two decades), `iters` conjugate-gradient
    iterations (tol 0: all run).  Each iteration streams O twice
    (16 M Pn bytes); the residual |S'delta - f| / |f| is checked with torch
    products on the device."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(7)
    base = torch.randn(M, Pn // 16, generator=g, device=dev, dtype=torch.float64)
    Ok = torch.randn(M, Pn, generator=g, device=dev, dtype=torch.float64)
    Ok += base.repeat(1, 16)
    Ok *= torch.logspace(-1, 1, Pn, device=dev, dtype=torch.float64)
    el = -5.0 + torch.randn(M, generator=g, device=dev, dtype=torch.float64) + 0.5 * Ok[:, 0]
    work = torch.empty((P.load().qmc_sr_workspace_size(M, Pn) + 7) // 8, dtype=torch.float64, device=dev)
    P.sr_step(Ok, el, eps, None, max_iter=2, tol=0.0, work=work)   # warm-up
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    P.sr_step(Ok, el, eps, None, max_iter=0, tol=0.0, work=work)
    e1.record()
    delta, f, res = P.sr_step(Ok, el, eps, None, max_iter=iters, tol=0.0, work=work)
    e2.record()
    torch.cuda.synchronize()
    t0, t1 = e0.elapsed_time(e1) / 1e3, e1.elapsed_time(e2) / 1e3
    t_iter = (t1 - t0) / iters
    Ob = Ok.mean(0)
    Sd = (Ok @ delta) / M
    Sp = Ok.t() @ Sd - Ob * (Ob @ delta) + eps * ((Ok - Ob) ** 2).mean(0) * delta
    chk = float((Sp - f).norm() / f.norm())
    bytes_iter = 16.0 * M * Pn
    return {"samples": M, "params": Pn, "eps": eps, "iterations": iters, "precision": "fp64",
            "moments_ms": round(1e3 * t0, 3), "ms_per_iteration": round(1e3 * t_iter, 4),
            "iteration_GBps": round(bytes_iter / t_iter / 1e9, 1),
            "iteration_frac_of_hbm_peak": round(bytes_iter / t_iter / 8e12, 3),
            "residual": float(f"{res.item():.3e}"), "residual_check": float(f"{chk:.3e}")}


def achievable_peaks():
    """Achievable peaks on this GPU beside the datasheet ones (best of 5): a
    STREAM-like 1 GiB copy (bytes read + written per second), a 1 GiB sum
    (read only, the proposal kernel's access pattern) and an 8192^3
    FP64 matrix product from the vendor library (flops per second).  These are
    measurement references only."""
    dev = torch.device("cuda:0")
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    best = float("inf")
    for _ in range(6):
        ev[0].record()
        b.copy_(a)
        ev[1].record()
        torch.cuda.synchronize()
        best = min(best, ev[0].elapsed_time(ev[1]))
    copy_gbs = 2 * n * 8 / (best * 1e-3) / 1e9
    acc = torch.empty((), dtype=torch.float64, device=dev)
    best = float("inf")
    for _ in range(6):
        ev[0].record()
        torch.sum(a, dim=0, out=acc)
        ev[1].record()
        torch.cuda.synchronize()
        best = min(best, ev[0].elapsed_time(ev[1]))
    read_gbs = n * 8 / (best * 1e-3) / 1e9
    del a, b
    m = 8192
    g = torch.Generator(device=dev).manual_seed(3)
    x = torch.randn(m, m, generator=g, dtype=torch.float64, device=dev)
    y = torch.randn(m, m, generator=g, dtype=torch.float64, device=dev)
    z = torch.empty_like(x)
    best = float("inf")
    for _ in range(6):
        ev[0].record()
        torch.matmul(x, y, out=z)
        ev[1].record()
        torch.cuda.synchronize()
        best = min(best, ev[0].elapsed_time(ev[1]))
    del x, y, z
    return {"hbm_copy_GBps": round(copy_gbs, 1), "hbm_read_GBps": round(read_gbs, 1), "fp64_gemm_TFLOPs": round(2 * m ** 3 / (best * 1e-3) / 1e12, 2),
            "datasheet": {"hbm_GBps": HBM_PEAK_GBS, "fp64_TFLOPs": 78.6, "fp32_TFLOPs": 157.3}}


def step_rooflines(s, Wk, precision, one, prop_roof, acc_model=None, p_rows=None, sweep_roof=None, rb_rows=None):
    """Roofline of each step of one evaluation (and the proposal) from the
    one-step timers: algorithmic bytes or flops per launch / average launch.
      basis:   writes the N x L values of every walker (FP64; FP32 in fp32 mode)
      P_build: 2 L^2 flops per basis row built, p_rows rows per walker (N,
               or n_dn when the up rows are reused; MFMA; FP64 but in fp32
               mode); the refined modes count the int8 operations of their 28
               digit products, 2 Lp^2 x 28 per row (Lp = L rounded up to 32)
      P_rebuild (fp64, fp32, mixed): the same per row over the rb_rows rows
               per walker rebuilt before the down electrons move (those of
               the up electrons that moved; n_up when not given)
      W_build: 2 n_up n_dn L flops per walker (FP64 MFMA accumulation)
      LU:      2 n^3 flops per walker per launch (FP64 vector ALU, latency-bound
               at n = 80: one workgroup per walker)
      Y_build: 2 x 2 n^2 L flops per walker (FP64 MFMA)
      sweep:   the persistent launch of a run of moves (FP64 and refined
               modes): the proposals' and fused accepts' algorithmic bytes
               (sweep_bytes) over its average launch; the proposal and accept
               entries then cover only the launches made on their own"""
    L, N, nu, nd = s.n_basis, s.n_up + s.n_dn, s.n_up, s.n_dn
    pr = N if p_rows is None else p_rows

    def p_model(rows):
        if precision in ("fp64", "fp32"):
            return ("mfma", 2.0 * L * L * rows * Wk, MFMA_PEAK_TFLOPS[precision], "TFLOP/s", 1e12)
        return ("mfma", 2.0 * ((L + 31) // 32 * 32) ** 2 * rows * Wk * OZ_DIGITS * (OZ_DIGITS + 1) // 2,
                INT8_PEAK_TOPS, "TOP/s", 1e12)
    models = {
        "basis": ("hbm", Wk * N * L * (4 if precision == "fp32" else 8), HBM_PEAK_GBS, "GB/s", 1e9),
        "P_build": p_model(pr),
        "W_build": ("mfma", 2.0 * nu * nd * L * Wk, 78.6, "TFLOP/s", 1e12),
        "LU": ("alu", 2.0 * nu ** 3 * Wk, 78.6, "TFLOP/s", 1e12),
        "Y_build": ("mfma", 4.0 * nu * nu * L * Wk, 78.6, "TFLOP/s", 1e12),
    }
    if precision in ("fp64", "fp32", "mixed"):
        models["P_rebuild"] = p_model(nu if rb_rows is None else rb_rows)
    out = {}
    for k, (bound, units, peak, unit, scale) in models.items():
        ms, cnt = one.get(k, (0.0, 0))
        if not cnt:
            continue
        avg = ms / cnt
        ach = units / (avg * 1e-3) / scale
        out[k] = {"bound": bound, "achieved": round(ach, 2), "peak": peak, "unit": unit,
                  "frac": round(ach / peak, 4), "avg_launch_us": round(avg * 1e3, 2)}
    keys = ("bound", "achieved", "peak", "unit", "frac", "avg_launch_us")
    if prop_roof is not None:
        out["propose"] = {k: prop_roof[k] for k in keys}
    if sweep_roof is not None:
        out["sweep"] = {k: sweep_roof[k] for k in keys + ("bytes_per_launch",)}
    if acc_model is not None and one.get("accept", (0.0, 0))[1] and sweep_roof is None:
        ms, cnt = one["accept"]
        avg = ms / cnt
        ach = acc_model / (avg * 1e-3) / 1e9
        out["accept"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(ach / HBM_PEAK_GBS, 4), "avg_launch_us": round(avg * 1e3, 2),
                         "bytes_per_launch": int(acc_model)}
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: the walker batch of one MI355X is the unit measured here; "
              "multi-GPU runs are not supported.", file=sys.stderr)
        sys.exit(2)
    import paper_2002_07401_amd as P
    from workloads import configs as C
    P.load()
    torch.cuda.set_device(0)
    if args.copy_probe_mib > 0:
        copy_probe(args.copy_probe_mib)
    w = C.mol_40nuc_160e(n_walkers=args.walkers)
    s = w.system
    N = s.n_up + s.n_dn
    main_prec = args.precision
    others = [p for p in PRECISIONS if p != main_prec]
    head = run_precision(P, C, w, args, main_prec)
    sides = {} if args.only else {p: run_precision(P, C, w, args, p) for p in others}
    res = {
        "metric": METRIC,
        "value": head["moves_per_s"],
        "unit": "walker-electron moves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed": "i8+f64", "mixed_fp32_rows": "i8+f32+f64", "bf16": "i8+bf16+f64",
                  "fp32": "f32+f64"}[main_prec],
        "data": "synthetic",
        "config": {"workload": "mol_40nuc_160e", "walkers": args.walkers, "electrons": N,
                   "basis": s.n_basis, "nuclei": len(s.Z), "refresh_every": s.refresh_every,
                   "precision": main_prec},
        "eloc_evals_per_s": head["eloc_evals_per_s"],
        "acceptance": head["acceptance"],
        "err_vs_oracle": head["err_vs_oracle"],
        "kernel_ms": head["kernel_ms"],
        "kernel_launches": head["kernel_launches"],
        "kernel_ms_one_step": head["kernel_ms_one_step"],
        "dominant_kernel": head["dominant_kernel"],
        "roofline": head["roofline"],
        "w_build_mfma": head["w_build_mfma"],
        "step_rooflines": head["step_rooflines"],
    }
    for p, rec in sides.items():
        res[p] = rec
    if main_prec == "fp64":
        for p, rec in sides.items():
            res[f"{p}_over_fp64_moves"] = round(rec["moves_per_s"] / head["moves_per_s"], 3)
            res[f"{p}_over_fp64_evals"] = round(rec["eloc_evals_per_s"] / head["eloc_evals_per_s"], 3)
    if not args.only:
        res["forces"] = forces_leg(P, C)
        res["multi_system"] = multi_leg(P, C)
        res["multi_system_bf16"] = multi_leg(P, C, precision="bf16")
        res["multi_system_refined"] = multi_leg(P, C, precision="mixed")
        res["large"] = large_leg(P, C)
        res["large_refined"] = large_leg(P, C, refined=True)
        res["large_refined_over_fp64_moves"] = round(res["large_refined"]["moves_per_s"] /
                                                     res["large"]["moves_per_s"], 3)
        res["large_refined_over_fp64_evals"] = round(res["large_refined"]["eloc_evals_per_s"] /
                                                     res["large"]["eloc_evals_per_s"], 3)
        res["lrdmc"] = lrdmc_leg(P, C)
        res["pfaffian"] = pfaffian_leg(P, C)
        res["sr"] = sr_leg(P)
        res["achievable_peaks"] = achievable_peaks()
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
