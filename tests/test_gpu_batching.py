"""A loop of one launch per k block reproduces the one-launch contractions (the batching study).

msgw_set_k_range restricts the split-precision pair-space polarization and self-energy (BF16 and
FP16 splits) to a range of k blocks (harness only); looping it over k must give the one-launch result
up to where the FP32 partial sums are flushed to FP64, and both must match the oracle.  Other paths
refuse a partial range, and a call that asks to reuse operands another op or q left in the scratch
is refused.
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


def _setup(torch, q, prec=2):
    import paper_1602_02313_amd as amd
    cfg = UNEVEN
    prob, run = make_run(cfg, precision=prec)
    M = torch.empty(int(run.mpre[q + 1] - run.mpre[q]), dtype=torch.complex64, device="cuda")
    run.ctx.synth_M(cfg.seed, q, 1, 1, amd.C64, M)
    run.green0(0.0)
    return cfg, prob, run, M


@pytest.mark.parametrize("prec", [2, 3])
@pytest.mark.parametrize("q", [0, 3])
def test_polarization_k_loop(torch, q, prec):
    import paper_1602_02313_amd as amd
    cfg, prob, run, M = _setup(torch, q, prec)
    NI, ntau = int(prob.ni[q]), prob.tau.size
    n = ntau * NI * NI
    run.ctx.polarization(q, 1, M, amd.C64, run.G_tau, prec, run.P_tau)
    P2 = torch.full((n,), float("nan"), dtype=torch.complex128, device="cuda")  # all written by the loop
    for k in range(cfg.nk):
        run.ctx.set_k_range(k, k + 1, reuse_prepared=k > 0)
        run.ctx.polarization(q, 1, M, amd.C64, run.G_tau, prec, P2)
    run.ctx.set_k_range()
    one = np_(run.P_tau[:n]).reshape(ntau, NI, NI)
    loop = np_(P2).reshape(ntau, NI, NI)
    g = gi.MGenerator(cfg)
    ref = o.polarization(g.q_blocks(q), oracle_G(prob), prob.kmq[q], cfg.scale)
    e_lo, e_ref = rel(loop, one), rel(loop, ref)
    print(f"q={q}: loop vs one launch {e_lo:.2e}, loop vs oracle {e_ref:.2e}")
    assert e_lo < 1e-6 and e_ref < 1e-5


@pytest.mark.parametrize("prec", [2, 3])
@pytest.mark.parametrize("q", [0, 3])
def test_self_energy_k_loop(torch, q, prec):
    import paper_1602_02313_amd as amd
    cfg, prob, run, M = _setup(torch, q, prec)
    NI, ntau = int(prob.ni[q]), prob.tau.size
    rng = np.random.default_rng(5 + q)
    X = rng.normal(size=(ntau, NI, NI)) + 1j * rng.normal(size=(ntau, NI, NI))
    W = (X + np.conj(np.swapaxes(X, 1, 2))) * 0.05 + np.eye(NI)[None]
    run.Wt_tau[:W.size].copy_(torch.from_numpy(W.ravel()))
    run.sig_tau.zero_()
    run.ctx.self_energy(q, 1, M, amd.C64, run.G_tau, run.Wt_tau, prec, run.sig_tau)
    one = np_(run.sig_tau).copy()
    run.sig_tau.zero_()
    for k in range(cfg.nk):
        run.ctx.set_k_range(k, k + 1, reuse_prepared=k > 0)
        run.ctx.self_energy(q, 1, M, amd.C64, run.G_tau, run.Wt_tau, prec, run.sig_tau)
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


def test_reuse_of_another_calls_operands_refused(torch):
    """P(k0) -> Sigma(k0) -> P(k1, reuse) would read Sigma's transposed M as g planes: the library
    refuses such a reuse (and a reuse across q ranges or precisions) on the host."""
    import paper_1602_02313_amd as amd
    cfg, prob, run, M = _setup(torch, 1)
    B = amd.BF16X3
    try:
        run.ctx.set_k_range(0, 1)
        run.ctx.polarization(1, 1, M, amd.C64, run.G_tau, B, run.P_tau)
        run.ctx.self_energy(1, 1, M, amd.C64, run.G_tau, run.Wt_tau, B, run.sig_tau)
        run.ctx.set_k_range(1, 2, reuse_prepared=True)
        with pytest.raises(amd.MsgwError) as e:
            run.ctx.polarization(1, 1, M, amd.C64, run.G_tau, B, run.P_tau)
        assert e.value.code == amd.EINVAL
        # the self-energy's own operands may be reused, but not for another precision
        run.ctx.self_energy(1, 1, M, amd.C64, run.G_tau, run.Wt_tau, B, run.sig_tau)
        with pytest.raises(amd.MsgwError) as e:
            run.ctx.self_energy(1, 1, M, amd.C64, run.G_tau, run.Wt_tau, amd.F16X3, run.sig_tau)
        assert e.value.code == amd.EINVAL
    finally:
        run.ctx.set_k_range()
    torch.cuda.synchronize()
