"""A loop of one launch per k block reproduces the one-launch contractions (the batching study).

msgw_set_k_range restricts the split-BF16 pair-space polarization and self-energy to a range of k
blocks (harness only); looping it over k must give the one-launch result up to where the FP32
partial sums are flushed to FP64, and both must match the oracle.  Other paths refuse a partial
range.
"""
import numpy as np
import pytest

import gwinputs as gi
import oracle as o
from gpu_util import make_run, np_, rel
from test_gpu_parity import UNEVEN, oracle_G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _setup(torch, q):
    import paper_1602_02313_amd as amd
    cfg = UNEVEN
    prob, run = make_run(cfg, precision=amd.BF16X3)
    M = torch.empty(int(run.mpre[q + 1] - run.mpre[q]), dtype=torch.complex64, device="cuda")
    run.ctx.synth_M(cfg.seed, q, 1, 1, amd.C64, M)
    run.green0(0.0)
    return cfg, prob, run, M


@pytest.mark.parametrize("q", [0, 3])
def test_polarization_k_loop(torch, q):
    import paper_1602_02313_amd as amd
    cfg, prob, run, M = _setup(torch, q)
    NI, ntau = int(prob.ni[q]), prob.tau.size
    n = ntau * NI * NI
    run.ctx.polarization(q, 1, M, amd.C64, run.G_tau, amd.BF16X3, run.P_tau)
    P2 = torch.full((n,), float("nan"), dtype=torch.complex128, device="cuda")  # all written by the loop
    for k in range(cfg.nk):
        run.ctx.set_k_range(k, k + 1, reuse_prepared=k > 0)
        run.ctx.polarization(q, 1, M, amd.C64, run.G_tau, amd.BF16X3, P2)
    run.ctx.set_k_range()
    one = np_(run.P_tau[:n]).reshape(ntau, NI, NI)
    loop = np_(P2).reshape(ntau, NI, NI)
    g = gi.MGenerator(cfg)
    ref = o.polarization(g.q_blocks(q), oracle_G(prob), prob.kmq[q], cfg.scale)
    e_lo, e_ref = rel(loop, one), rel(loop, ref)
    print(f"q={q}: loop vs one launch {e_lo:.2e}, loop vs oracle {e_ref:.2e}")
    assert e_lo < 1e-6 and e_ref < 1e-5


@pytest.mark.parametrize("q", [0, 3])
def test_self_energy_k_loop(torch, q):
    import paper_1602_02313_amd as amd
    cfg, prob, run, M = _setup(torch, q)
    NI, ntau = int(prob.ni[q]), prob.tau.size
    rng = np.random.default_rng(5 + q)
    X = rng.normal(size=(ntau, NI, NI)) + 1j * rng.normal(size=(ntau, NI, NI))
    W = (X + np.conj(np.swapaxes(X, 1, 2))) * 0.05 + np.eye(NI)[None]
    run.Wt_tau[:W.size].copy_(torch.from_numpy(W.ravel()))
    run.sig_tau.zero_()
    run.ctx.self_energy(q, 1, M, amd.C64, run.G_tau, run.Wt_tau, amd.BF16X3, run.sig_tau)
    one = np_(run.sig_tau).copy()
    run.sig_tau.zero_()
    for k in range(cfg.nk):
        run.ctx.set_k_range(k, k + 1, reuse_prepared=k > 0)
        run.ctx.self_energy(q, 1, M, amd.C64, run.G_tau, run.Wt_tau, amd.BF16X3, run.sig_tau)
    run.ctx.set_k_range()
    loop = np_(run.sig_tau)
    g = gi.MGenerator(cfg)
    ref = o.sigma_c(g.q_blocks(q), oracle_G(prob), prob.kmq[q], W, cfg.scale)
    e_lo, e_ref = rel(loop, one), rel(loop, ref)
    print(f"q={q}: loop vs one launch {e_lo:.2e}, loop vs oracle {e_ref:.2e}")
    assert e_lo < 1e-6 and e_ref < 1e-5


def test_partial_range_refused_elsewhere(torch):
    import paper_1602_02313_amd as amd
    cfg, prob, run, M = _setup(torch, 1)
    run.ctx.set_k_range(1, 2)
    try:
        for prec, variant in ((amd.BF16X3, len(run.ctx.variants(0, amd.BF16X3)) - 1), (amd.FP32, 0)):
            run.ctx.set_variant(0, prec, variant)
            with pytest.raises(amd.MsgwError):
                run.ctx.polarization(1, 1, M, amd.C64, run.G_tau, prec, run.P_tau)
            run.ctx.set_variant(0, prec, 0)
        with pytest.raises(amd.MsgwError):
            run.ctx.set_k_range(2, 2)
    finally:
        run.ctx.set_k_range()
    torch.cuda.synchronize()
