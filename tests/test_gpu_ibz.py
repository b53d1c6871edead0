"""GPU: the irreducible-wedge reduction (Sec. III.C) against the full zone and the oracle.

Cubic-symmetric inputs (gwinputs.CubicGenerator; on the device msgw_synth_M_cubic, checked against
it): on a 3 x 3 x 3 grid the library computes P, W~ and the contractions for the 4 irreducible q
instead of 27 and adds their contributions over the stars (msgw_sigma_star).  Sigma^c(tau) and
Sigma^x must match the full-zone pass of the same library and the oracle's full-zone sums: rel 1e-10
in FP64, 1e-6 for the split-FP16 contractions.
"""
import numpy as np
import pytest

import gwinputs as gi
import oracle as o
from gpu_util import check, np_, rel

pytestmark = pytest.mark.gpu

CUB = gi.Config(name="cub3", grid=(3, 3, 3), bands=((3, -1.0, -0.1), (3, 0.1, 1.5)), nb=6, ni=33,
                ntau=20, mesh="upm", beta=20.0, niw_f=16, niw_b=16)


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def cub_oracle():
    cfg = CUB
    prob = gi.make_cubic_problem(cfg)
    gen = gi.CubicGenerator(cfg)
    G = o.green0(prob.eps, prob.nb, prob.tau, cfg.beta)
    occ = -G[:, :, -1]
    sc = sx = 0
    for q in range(cfg.nk):
        Mq = gen.q_blocks(q)
        P = o.polarization(Mq, G, prob.kmq[q], cfg.scale)
        _, R = o.screen(o.tau_to_iw(P, prob.tau, cfg.beta, o.BOSON, cfg.niw_b), prob.v[q])
        Wt = o.wt_tau(R, P, prob.v[q], prob.tau, cfg.beta)
        sc = sc + o.sigma_c(Mq, G, prob.kmq[q], Wt, cfg.scale)
        sx = sx + o.sigma_x(Mq, occ, prob.kmq[q], prob.v[q], cfg.scale)
    return cfg, prob, gen, sc, sx


def _run(cfg, prob, precision):
    import paper_1602_02313_amd as amd
    return amd.GWRun(cfg.nk, prob.kmq, prob.nb, prob.ni, prob.tau, cfg.beta, cfg.niw_f, cfg.niw_b, cfg.scale,
                     prob.eps, prob.v, prob.n_target, precision=precision, q_batch=1)


def test_synth_cubic_matches_host_generator(torch, cub_oracle):
    import paper_1602_02313_amd as amd
    cfg, prob, gen, _, _ = cub_oracle
    run = _run(cfg, prob, amd.FP64)
    ref = np.concatenate([gen.q_packed(q) for q in range(cfg.nk)])
    for dt, ct in ((amd.C128, torch.complex128), (amd.C64, torch.complex64)):
        buf = torch.empty(ref.size, dtype=ct, device="cuda")
        run.ctx.synth_M_cubic(cfg.seed, 0, cfg.nk, dt, buf)
        torch.cuda.synchronize()
        got = np_(buf)
        tol = 1e-14 if dt == amd.C128 else 1e-6
        assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("prec", [0, 3])
def test_ibz_pass_matches_full_zone_and_oracle(torch, cub_oracle, prec):
    import paper_1602_02313_amd as amd
    cfg, prob, gen, sc_ref, sx_ref = cub_oracle
    src = amd.SynthCubicM(cfg.seed)
    full = _run(cfg, prob, prec)
    full.green0(0.0)
    full.sigma_pass(src)
    red = _run(cfg, prob, prec)
    red.set_symmetry(gen.rot_k)
    assert red.ibz == [q for q, _ in o.ibz_stars(gen.rot_k)] and sum(red.star_size) == cfg.nk
    print(f"\nirreducible q {red.ibz} (stars {red.star_size}): {len(red.ibz)} of {cfg.nk}")
    red.green0(0.0)
    red.sigma_pass(src)
    torch.cuda.synchronize()
    gate = 1e-10 if prec == 0 else 1e-6
    check(f"IBZ Sigma^c prec={prec} vs oracle", np_(red.sig_tau), sc_ref, gate, -1)
    assert rel(np_(red.sig_x), sx_ref) < gate
    # the same library's full-zone pass
    e = rel(np_(red.sig_tau), np_(full.sig_tau))
    print(f"IBZ vs full zone (library): rel {e:.2e}")
    assert e < gate
    assert rel(np_(red.sig_x), np_(full.sig_x)) < gate
    if prec != 0:
        # at this (unphysical) scale |Sigma^x| ~ 1e3 Ha: the split precision's 1e-6 of it moves the energies
        # of G by ~1e-3 Ha, which exp(-E tau) amplifies; the FP64 case checks G and the gap
        return
    # and through the transform, a Dyson step at a fixed mu and the gap
    for r in (full, red):
        r.sigma_to_iw()
        r.mu.zero_()
        r.dyson(False)
        r.gap()
    torch.cuda.synchronize()
    assert rel(np_(red.G_tau), np_(full.G_tau)) < gate
    assert abs(red.gap_d.item() - full.gap_d.item()) < 1e-6


def test_symmetry_validation(torch, cub_oracle):
    import paper_1602_02313_amd as amd
    cfg, prob, gen, _, _ = cub_oracle
    run = _run(cfg, prob, amd.FP64)
    C = torch.zeros_like(run.sig_tau)
    with pytest.raises(amd.MsgwError) as e:           # no symmetry set
        run.ctx.sigma_star(0, C, None, run.sig_tau, None)
    assert e.value.code == amd.EINVAL
    bad = gen.rot_k.copy()
    bad[3, [1, 2]] = bad[3, [2, 1]]                    # breaks R (k - q) = R k - R q
    with pytest.raises(amd.MsgwError) as e:
        run.ctx.set_symmetry(bad)
    assert e.value.code == amd.EINVAL
    run.ctx.set_symmetry(gen.rot_k)
    ibz, st = run.ctx.ibz()
    non_ibz = next(q for q in range(cfg.nk) if q not in ibz)
    with pytest.raises(amd.MsgwError) as e:
        run.ctx.sigma_star(non_ibz, C, None, run.sig_tau, None)
    assert e.value.code == amd.EINVAL
    with pytest.raises(amd.MsgwError) as e:            # NI = 32 closes no shell
        cfg2 = CUB.replace(ni=32)
        prob2 = gi.make_problem(cfg2)
        run2 = _run(cfg2, prob2, amd.FP64)
        buf = torch.empty(int(run2.mpre[1]), dtype=torch.complex128, device="cuda")
        run2.ctx.synth_M_cubic(1, 0, 1, amd.C128, buf)
    assert e.value.code == amd.ESHAPE
