"""Host logic of bench.py (no GPU): the dense flop model and the use of the counter record."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import gwinputs as gi  # noqa: E402


def test_flop_model_closed_form():
    """Uniform band counts and basis sizes: F_P = 8 NI^2 Nb^2 Ntau Nk^2 and F_Sigma adds the
    8 NI Nb^2 Ntau Nk^2 of the final dot products."""
    for cfg in (gi.C1, gi.C2):
        prob = gi.make_problem(cfg)
        nb, ni, nt, nk = int(prob.nb[0]), int(prob.ni[0]), prob.tau.size, cfg.nk
        assert np.all(prob.nb == nb) and np.all(prob.ni == ni)
        fp, fs = bench.flop_model(prob)
        assert fp == 8.0 * ni * ni * nb * nb * nt * nk * nk
        assert fs == fp + 8.0 * ni * nb * nb * nt * nk * nk


def test_flop_model_uneven_counts():
    """Uneven band counts: the sum over (q, k) of 8 NI_q^2 Nb_k Nb_{k-q} Ntau, on a small grid."""
    cfg = gi.C4.replace(grid=(2, 2, 2), name="c4_small_grid")
    prob = gi.make_problem(cfg)
    assert len(set(int(x) for x in prob.nb)) > 1 and len(set(int(x) for x in prob.ni)) > 1
    fp, _ = bench.flop_model(prob)
    ref = sum(8.0 * int(prob.ni[q]) ** 2 * int(prob.nb[k]) * int(prob.nb[prob.kmq[q, k]]) * prob.tau.size
              for q in range(cfg.nk) for k in range(cfg.nk))
    assert fp == ref


def test_counter_record_is_used_only_when_it_matches():
    """The committed record matches its kernel source; any other workload, precision, q batch or
    tile gives no record."""
    path = os.path.join(ROOT, "profiles", "traffic_c2_bf16x3.json")
    with open(path) as f:
        rec = json.load(f)
    import hashlib
    qb = rec["q_batch"]
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        current = hashlib.sha256(f.read()).hexdigest() == rec["source_sha256"]
    for kernel, k in rec["kernels"].items():
        got = bench.measured_record(kernel, k["tile"], "bf16x3", "c2_k64_nb64_ni400", qb)
        if not current:  # the kernel source changed since the counters were taken
            assert got is None
            continue
        assert got is not None and got["traffic_bytes"] == k["traffic_bytes"]
        assert bench.measured_record(kernel, k["tile"], "fp32", "c2_k64_nb64_ni400", qb) is None
        assert bench.measured_record(kernel, k["tile"], "bf16x3", "c1_k8_nb16_ni64", qb) is None
        assert bench.measured_record(kernel, k["tile"], "bf16x3", "c2_k64_nb64_ni400", qb + 1) is None
        assert bench.measured_record(kernel, k["tile"] + " other", "bf16x3", "c2_k64_nb64_ni400", qb) is None
