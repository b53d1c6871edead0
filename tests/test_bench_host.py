"""Host logic of bench.py (no GPU): the flop models, the iteration slicing and the counter record."""
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


def test_executed_mfma_model_closed_form():
    """Uniform shapes, 16-row polarization blocks: ceil(NI/16)(ceil(NI/16)+1)/2 working blocks of
    8 waves x (N_k K_pad / 16) steps x 6 MFMAs per 32-wide tau tile; the self-energy: N_k ceil(K/512)
    chunks of 8 waves x (8x8-pair upper-triangle blocks) x 8 steps x 6 MFMAs per tau tile."""
    cfg = gi.C5
    prob = gi.make_problem(cfg)
    NI, nb, nk, ntau = int(prob.ni[0]), int(prob.nb[0]), cfg.nk, prob.tau.size
    K = nb * nb
    tiles = -(-ntau // 32)
    b16 = -(-NI // 16)
    want_p = b16 * (b16 + 1) // 2 * 8 * (nk * (-(-K // 64) * 64) // 16) * 6 * tiles * 32768
    got_p = bench.executed_mfma_flops(prob, 0, "pair-space 16x16 pairs K64 st4x8 3-buffer", 0, 1)
    assert got_p == want_p
    b8 = -(-NI // 8)
    want_s = nk * (-(-K // 512)) * 8 * (b8 * (b8 + 1) // 2) * 8 * 6 * tiles * 32768
    for name in bench.SIGZ_NAMES:  # the static grid and the persistent queue execute the same items
        assert bench.executed_mfma_flops(prob, 1, name, 0, 1) == want_s
    assert bench.executed_mfma_flops(prob, 0, "pair-space 16x16 pairs K64 3-buffer persistent LPT queue", 0, 1) == got_p
    # two q cost twice one; a tile form has no model
    assert bench.executed_mfma_flops(prob, 1, bench.SIGZ_NAMES[0], 3, 2) == 2 * want_s
    assert bench.executed_mfma_flops(prob, 0, "WI2 WJ2 T2", 0, 1) is None
    # the executed 16-bit work against the dense count of the flop model: about 3 x 3/4 (three split
    # products, real weight against complex pairs of the upper triangle) plus tau padding
    fp, fs = bench.flop_model(prob, qs=[0])
    assert 0.8 < got_p / fp < 1.0 and 0.8 < want_s / fs < 1.0


def test_iteration_slices_and_batches():
    for nk, steps in ((125, 20), (64, 20), (8, 3), (125, 125), (7, 1)):
        sl = bench.iteration_slices(nk, steps)
        assert len(sl) == steps and sl[0][0] == 0 and sl[-1][1] == nk
        assert all(a < b for a, b in sl) and all(sl[i][1] == sl[i + 1][0] for i in range(steps - 1))
        for a, b in sl:
            for qmax in (1, 3, 8):
                bs = bench.sub_batches(a, b, qmax)
                assert bs[0][0] == a and sum(n for _, n in bs) == b - a
                assert all(1 <= n <= qmax for _, n in bs)
                assert max(n for _, n in bs) - min(n for _, n in bs) <= 1


def test_traffic_record_is_used_only_when_it_matches(tmp_path):
    import hashlib
    src = os.path.join("paper_1602_02313_amd", "csrc", "k_mfma.hip")
    with open(os.path.join(ROOT, src), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    rec = {"workload": "c5_k125_nb128_ni700_scgw", "precision": "f16x3", "source": src,
           "source_sha256": sha, "kernels": {"polarization": {"tile": "t", "bytes_per_q": 5.0}}}
    path = tmp_path / "rec.json"
    path.write_text(json.dumps(rec))
    ok = bench.traffic_record("polarization", "t", "f16x3", "c5_k125_nb128_ni700_scgw", str(path))
    assert ok is not None and ok["bytes_per_q"] == 5.0
    assert bench.traffic_record("polarization", "t", "bf16x3", "c5_k125_nb128_ni700_scgw", str(path)) is None
    assert bench.traffic_record("polarization", "u", "f16x3", "c5_k125_nb128_ni700_scgw", str(path)) is None
    assert bench.traffic_record("self_energy", "t", "f16x3", "c5_k125_nb128_ni700_scgw", str(path)) is None
    assert bench.traffic_record("polarization", "t", "f16x3", "c2_k64_nb64_ni400", str(path)) is None
    rec["source_sha256"] = "0" * 64                     # the kernel source changed since the counters
    path.write_text(json.dumps(rec))
    assert bench.traffic_record("polarization", "t", "f16x3", "c5_k125_nb128_ni700_scgw", str(path)) is None
