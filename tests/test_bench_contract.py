"""The benchmark's contract on the CPU: one GPU only (a request for more
exits with status 2 before any device work), and the algorithmic counts the
rooflines are priced with.

Proposal kernel (the streaming part of a single-electron move): every walker
reads the n_other x L rows of the opposite spin (esz bytes each), psi(r') (8 L)
and the moved electron's inverse column (8 n), and writes the new W row (8 n).
The evaluation's P = Phi Lambda product costs 2 L^2 flops per basis row over
all N rows.
"""
import os
import subprocess
import sys

import bench
from workloads import configs as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=300)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout.strip() == ""


def test_algorithmic_counts_160e():
    s = C.mol_40nuc_160e(n_walkers=4).system
    Wk, L, n, N = 1024, 600, 80, 160
    m = bench.kernel_models(s, Wk, 8, 0.74)
    assert m["propose"] == ("hbm", Wk * (8 * n * L + 8 * L + 16 * n))
    assert m["propose"][1] == 399_441_920
    assert m["P_build"] == ("mfma", 2.0 * L * L * Wk * N)
    # FP32 and BF16 rows halve and quarter the streamed rows only
    assert bench.kernel_models(s, Wk, 4, 0.74)["propose"][1] == Wk * (4 * n * L + 8 * L + 16 * n)
    assert bench.kernel_models(s, Wk, 2, 0.74)["propose"][1] == Wk * (2 * n * L + 8 * L + 16 * n)


def test_step_rooflines_arithmetic():
    s = C.mol_40nuc_160e(n_walkers=4).system
    one = {"basis": (0.5, 1), "P_build": (3.0, 1), "W_build": (0.4, 1), "LU": (1.8, 6), "Y_build": (0.8, 1)}
    prop = {"bound": "hbm", "achieved": 6000.0, "peak": 8000.0, "unit": "GB/s", "frac": 0.75, "avg_launch_us": 66.6}
    r = bench.step_rooflines(s, 1024, "fp64", one, prop)
    L, N, n = 600, 160, 80
    assert abs(r["basis"]["achieved"] - 1024 * N * L * 8 / 0.5e-3 / 1e9) < 0.01
    assert abs(r["P_build"]["achieved"] - 2.0 * L * L * N * 1024 / 3.0e-3 / 1e12) < 0.01
    assert abs(r["LU"]["achieved"] - 2.0 * n ** 3 * 1024 / 0.3e-3 / 1e12) < 0.01
    assert r["propose"]["frac"] == 0.75


def test_screened_and_refined_counts_160e():
    """Screened proposals (QMC_REFINED) stream only the kept basis functions:
    kept columns of n FP64 values plus their index and value (12 bytes each),
    the inverse column and the new row (16 n).  The refined products count the
    int8 operations of the 28 digit products (7 digits per FP64 row, pairs
    a + b < 7) over L rounded up to 32 (608 at L = 600)."""
    s = C.mol_40nuc_160e(n_walkers=4).system
    Wk, L, n, N = 1024, 600, 80, 160
    m = bench.kernel_models(s, Wk, 8, 0.74, kept=144.0)
    assert m["propose"] == ("hbm", Wk * (144.0 * (8 * n + 12) + 16 * n))
    one = {"P_build": (2.0, 1)}
    prop = {"bound": "hbm", "achieved": 1.0, "peak": 8000.0, "unit": "GB/s", "frac": 0.0, "avg_launch_us": 1.0}
    r = bench.step_rooflines(s, Wk, "mixed", one, prop)
    ops = 2.0 * 608 * 608 * N * Wk * 28
    assert r["P_build"]["unit"] == "TOP/s" and r["P_build"]["peak"] == 5000.0
    assert abs(r["P_build"]["achieved"] - ops / 2.0e-3 / 1e12) < 0.01


def test_p_rows_of_evaluations_at_current_positions_160e():
    """After a full sweep the up rows of P are current (rebuilt before the down
    electrons moved): the evaluation's P_build is priced on the n_dn = 80 rows
    per walker it builds, the rebuild on the n_up = 80 rows."""
    s = C.mol_40nuc_160e(n_walkers=4).system
    Wk, L, n = 1024, 600, 80
    assert bench.kernel_models(s, Wk, 8, 0.74, p_rows=n)["P_build"] == ("mfma", 2.0 * L * L * Wk * n)
    one = {"P_build": (1.5, 1), "P_rebuild": (1.5, 1)}
    prop = {"bound": "hbm", "achieved": 1.0, "peak": 8000.0, "unit": "GB/s", "frac": 0.0, "avg_launch_us": 1.0}
    r = bench.step_rooflines(s, Wk, "fp64", one, prop, p_rows=n)
    assert abs(r["P_build"]["achieved"] - 2.0 * L * L * n * Wk / 1.5e-3 / 1e12) < 0.01
    assert abs(r["P_rebuild"]["achieved"] - r["P_build"]["achieved"]) < 1e-9
    r = bench.step_rooflines(s, Wk, "mixed", one, prop, p_rows=n)
    assert abs(r["P_build"]["achieved"] - 2.0 * 608 * 608 * n * Wk * 28 / 1.5e-3 / 1e12) < 0.01
