"""GPU parity of the FULL band-matrix self-energy in split FP16 (MSGW_SIGMA_FULL with MSGW_F16X3): the
F16X3 product W~ M and the FP64 contraction with conj(M) G against the oracle's sigma_c(full=True),
gate rel 1e-6 (the split path's tolerance on Sigma), with the worst tau slice and the largest
absolute error bounded as in the other mixed-precision tests.

Shapes: the small, uneven and 133-row cases of the DIAG tests (tau chunks of 8 with a ragged last
one), and a case with 70 bands and NI = 150 whose products span several 64 x 128 tiles of W~ M with
ragged edges and two 64-band tiles of Sigma_nn' per k.
"""
import numpy as np
import pytest

import gwinputs as gi
import oracle as o
from gpu_util import check, make_run, np_, rel
from test_gpu_parity import SMALL, TILES, UNEVEN, _oracle_pw, oracle_G

pytestmark = pytest.mark.gpu

GATE = 1e-6
BANDS = gi.tiny(name="bands70", grid=(2, 1, 1), nocc=30, nemp=40, ni=150, ntau=12, beta=8.0, niw=12)


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("cfg", [SMALL, UNEVEN, TILES, BANDS])
def test_self_energy_full_f16x3(torch, cfg):
    import paper_1602_02313_amd as amd
    prob, run = make_run(cfg, precision=amd.F16X3, sigma_mode=amd.SIGMA_FULL)
    g = gi.MGenerator(cfg)
    G = oracle_G(prob)
    run.green0(0.0)
    run.sig_tau.zero_()
    print(f"\n[{cfg.name}] FULL F16X3: nb {list(prob.nb)}, NI {list(prob.ni)}, {prob.tau.size} tau", flush=True)
    ref = 0
    for q in range(cfg.nk):
        _, _, _, _, Wt = _oracle_pw(prob, g, q, G)
        run.Wt_tau[:Wt.size].copy_(torch.from_numpy(Wt.ravel()))
        M = torch.from_numpy(g.q_packed(q).astype(np.complex64)).to("cuda")
        run.ctx.self_energy(q, 1, M, amd.C64, run.G_tau, run.Wt_tau, amd.F16X3, run.sig_tau)
        ref = ref + o.sigma_c(g.q_blocks(q), G, prob.kmq[q], Wt, cfg.scale, full=True)
    torch.cuda.synchronize()
    got = np_(run.sig_tau)
    check(f"Sigma FULL {cfg.name} F16X3", got, ref, GATE, -1)
    # rows and columns past each k's bands stay untouched
    for k in range(cfg.nk):
        nb = int(prob.nb[k])
        assert (got[k, nb:] == 0).all() and (got[k, :, nb:] == 0).all()


def test_full_f16x3_pass_matches_fp64(torch):
    """A whole FULL sigma pass (P, screen, W~(tau), Sigma^c_nn', Sigma^x_nn') in F16X3 against the same
    pass in FP64, q batched."""
    import paper_1602_02313_amd as amd
    cfg = SMALL
    g = gi.MGenerator(cfg)
    out = {}
    for prec, mdt in ((amd.FP64, amd.C128), (amd.F16X3, amd.C64)):
        prob, run = make_run(cfg, precision=prec, sigma_mode=amd.SIGMA_FULL, q_batch=cfg.nk)
        run.green0(0.0)
        run.sigma_pass(amd.HostM(lambda q: g.q_packed(q), mdt))
        torch.cuda.synchronize()
        out[prec] = (np_(run.sig_tau).copy(), np_(run.sig_x).copy())
    (c64_, x64_), (c16, x16) = out[amd.FP64], out[amd.F16X3]
    check("FULL pass Sigma^c F16X3 vs FP64", c16, c64_, GATE, -1)
    ex = rel(x16, x64_)
    print(f"FULL pass Sigma^x F16X3 vs FP64: rel {ex:.2e}")
    assert ex < GATE


def test_full_mode_refuses_other_split_precisions(torch):
    import paper_1602_02313_amd as amd
    cfg = SMALL
    prob, run = make_run(cfg, precision=amd.BF16X3, sigma_mode=amd.SIGMA_FULL)
    g = gi.MGenerator(cfg)
    M = torch.from_numpy(g.q_packed(0).astype(np.complex64)).to("cuda")
    with pytest.raises(amd.MsgwError) as e:
        run.ctx.self_energy(0, 1, M, amd.C64, run.G_tau, run.Wt_tau, amd.BF16X3, run.sig_tau)
    assert e.value.code == amd.ENOTSUP
