"""The large workloads at full size, one q each, sampled against the FP64 oracle.

Three shapes, each run for one q in the launch configuration of the bench (one q per launch, default
tile variants):
  * 6x6x6 k-points, 128 bands (24 semicore, 40 valence, 64 empty), NI = 800, 121 tau points;
  * the same k-mesh with per-k band counts drawn from [96, 160] and per-q NI from [500, 900]
    (the q with the largest NI, so the largest blocks of the workload);
  * 5x5x5 k-points, 128 bands, NI = 700, 161 tau points (two 96-wide tau chunks, ragged).
Compared entry by entry:
  * P_IJ(q, tau) on sampled (tau, I, J), covering both triangles, the diagonal, tile edges and the
    last row I = NI - 1 (split FP16, split BF16 and FP32 on every shape);
  * this q's contribution to Sigma^c_n(k, tau) for two k and three tau, with a synthetic Hermitian
    W~(tau) of the decaying profile of a screened interaction;
  * the FP64 screen at full NI on a synthetic negative-definite P(i nu): W~(i nu) on four
    frequencies and W~(tau) on a square index subset at five tau points.
Gates: P and Sigma^c relative error <= 1e-6 (the split-precision tolerance on Sigma, for every
precision at these sizes), with the worst tau slice and the max-abs error within 10x; the FP64 screen
<= 1e-10.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import gwinputs as gi
import oracle as o
from gpu_util import check, np_, rel

pytestmark = pytest.mark.gpu

GATE = 1e-6


def _pick_q(cfg):
    ni = gi.basis_sizes(cfg)
    return int(np.argmax(ni)) if cfg.ni is None else 1


SHAPES = {"k216_nb128_ni800": gi.C3, "k216_uneven": gi.C4, "k125_nb128_ni700_ntau161": gi.C5}


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module", params=list(SHAPES))
def big(request, torch):
    import paper_1602_02313_amd as amd
    cfg = SHAPES[request.param]
    q = _pick_q(cfg)
    prob = gi.make_problem(cfg)
    run = amd.GWRun(cfg.nk, prob.kmq, prob.nb, prob.ni, prob.tau, cfg.beta, cfg.niw_f, cfg.niw_b,
                    cfg.scale, prob.eps, prob.v, prob.n_target, precision=amd.BF16X3, q_batch=1)
    M = torch.empty(int(run.mpre[q + 1] - run.mpre[q]), dtype=torch.complex64, device="cuda")
    print(f"\n[{cfg.name}] q={q} NI={prob.ni[q]} M {M.numel() * 8 / 1e9:.1f} GB", flush=True)
    run.ctx.synth_M(cfg.seed, q, 1, 1, amd.C64, M)
    run.green0(0.0)
    torch.cuda.synchronize()
    yield cfg, q, prob, run, M
    del M, run
    torch.cuda.empty_cache()


def _sample(NI, seed, n):
    rng = np.random.default_rng(seed)
    edges = [0, 15, 16, 31, 32, 63, 64, NI - 1]
    return np.unique(np.concatenate([edges, rng.choice(NI, n, replace=False)]))


def _host_blocks(cfg, q, rows=None, ks=None):
    g = gi.MGenerator(cfg)
    ks = range(cfg.nk) if ks is None else ks
    with ThreadPoolExecutor(8) as ex:
        return dict(zip(ks, ex.map(lambda k: g.block(q, k, rows=rows), ks)))


def _G(prob):
    return o.green0(prob.eps, prob.nb, prob.tau, prob.cfg.beta, 0.0)


@pytest.mark.parametrize("prec", [3, 2, 1])
def test_polarization_sampled(torch, big, prec):
    import paper_1602_02313_amd as amd
    cfg, q, prob, run, M = big
    print(f"\n[{cfg.name}] polarization prec={prec}", flush=True)
    NI, ntau = int(prob.ni[q]), prob.tau.size
    run.ctx.polarization(q, 1, M, amd.C64, run.G_tau, prec, run.P_tau)
    rows = _sample(NI, 10 + q, 6)
    cols = np.unique(np.concatenate([rows[::2], _sample(NI, 20 + q, 6)]))
    taus = np.array(sorted({0, 1, ntau // 2, 95, 96, ntau - 2, ntau - 1}))
    Pd = run.P_tau[:ntau * NI * NI].view(ntau, NI, NI)
    ti, ri, ci = (torch.from_numpy(a).to("cuda") for a in (taus, rows, cols))
    got = np_(Pd[ti][:, ri][:, :, ci])
    sel = np.union1d(rows, cols)
    blocks = _host_blocks(cfg, q, rows=sel)
    ref = o.polarization([blocks[k] for k in range(cfg.nk)], _G(prob), prob.kmq[q], cfg.scale,
                         taus=taus, rows=np.searchsorted(sel, rows), cols=np.searchsorted(sel, cols))
    check(f"[{cfg.name}] P prec={prec} ({got.size} entries)", got, ref, GATE, 0)


def _synthetic_W(cfg, NI, ntau, tau, seed):
    """Hermitian W~(tau) = f(tau) A + g(tau) B with a decaying-in-I profile."""
    rng = np.random.default_rng(seed)
    d = 1.0 / (1.0 + np.arange(NI) / 16.0)
    sd = np.sqrt(d)

    def herm(scale):
        X = (rng.normal(size=(NI, NI)) + 1j * rng.normal(size=(NI, NI))) * scale
        return (X + X.conj().T) * sd[:, None] * sd[None, :]

    A = herm(0.01) + np.diag(5.0 * d)
    B = herm(0.02)
    x = tau / cfg.beta
    f = np.exp(-8.0 * x) + np.exp(-8.0 * (1.0 - x))
    g = np.cos(2.0 * np.pi * x)
    return f[:, None, None] * A[None] + g[:, None, None] * B[None]


@pytest.mark.parametrize("prec", [3, 2, 1])
def test_self_energy_sampled(torch, big, prec):
    import paper_1602_02313_amd as amd
    cfg, q, prob, run, M = big
    print(f"\n[{cfg.name}] self-energy prec={prec}", flush=True)
    NI, ntau = int(prob.ni[q]), prob.tau.size
    W = _synthetic_W(cfg, NI, ntau, prob.tau, 3 + q)
    run.Wt_tau[:W.size].copy_(torch.from_numpy(W.ravel()))
    run.sig_tau.zero_()
    run.ctx.self_energy(q, 1, M, amd.C64, run.G_tau, run.Wt_tau, prec, run.sig_tau)
    ks = [0, cfg.nk // 2 + 1]
    taus = [0, ntau // 2, ntau - 1]
    got = np_(run.sig_tau)[np.ix_(ks, np.arange(run.sig_tau.shape[1]), taus)]
    blocks = _host_blocks(cfg, q, ks=ks)
    Mq = [blocks.get(k) for k in range(cfg.nk)]
    ref = o.sigma_c(Mq, _G(prob), prob.kmq[q], W, cfg.scale, taus=taus, ks=ks)
    check(f"[{cfg.name}] Sigma^c prec={prec}", got, ref, GATE, -1)


def test_screen_full_ni(torch, big):
    """FP64 screen and W~(tau) at the full NI of the shape, synthetic P."""
    cfg, q, prob, run, M = big
    NI, ntau, niw = int(prob.ni[q]), prob.tau.size, cfg.niw_b
    rng = np.random.default_rng(40 + q)
    d = 1.0 / (1.0 + np.arange(NI) / 16.0)
    B = (rng.normal(size=(NI, NI)) + 1j * rng.normal(size=(NI, NI))) * np.sqrt(d)[:, None]
    P0 = -(B @ B.conj().T) / NI * 0.02                  # negative definite, like P(i nu)
    C = rng.normal(size=(NI, NI)) + 1j * rng.normal(size=(NI, NI))
    P1 = (C + C.conj().T) * 1e-4
    nu = o.matsubara(o.BOSON, niw, cfg.beta)
    lor = 1.0 / (1.0 + (nu / 0.5) ** 2)
    Piw = lor[:, None, None] * P0[None] + (lor ** 2)[:, None, None] * P1[None]
    x = prob.tau / cfg.beta
    Ptau = (np.exp(-6.0 * x) + np.exp(-6.0 * (1.0 - x)))[:, None, None] * P0[None]
    run.P_iw[:Piw.size].copy_(torch.from_numpy(Piw.ravel()))
    run.P_tau[:Ptau.size].copy_(torch.from_numpy(Ptau.ravel()))
    vq = torch.from_numpy(np.asarray(prob.v[q], dtype=np.float64)).to("cuda")
    run.ctx.screen(q, 1, run.P_iw, vq, run.Wt_iw, run.R_iw, run.info)
    run.ctx.screened_tau(q, 1, run.R_iw, run.P_tau, vq, run.Wt_tau)
    torch.cuda.synchronize()
    assert int(run.info[:niw].abs().max()) == 0
    W, R = o.screen(Piw, prob.v[q])
    nus = [0, 1, niw // 2, niw - 1]
    Wg = run.Wt_iw[:Piw.size].view(niw, NI, NI)
    e_w = rel(np_(Wg[nus]), W[nus])
    S = _sample(NI, 50 + q, 10)
    taus = [0, 1, ntau // 2, ntau - 2, ntau - 1]
    sub = np.ix_(np.arange(niw), S, S)
    Wt_ref = o.wt_tau(R[sub], Ptau[np.ix_(np.arange(ntau), S, S)], np.asarray(prob.v[q])[S],
                      prob.tau, cfg.beta)[taus]
    Wtg = run.Wt_tau[:Ptau.size].view(ntau, NI, NI)
    Si = torch.from_numpy(S).to("cuda")
    got_t = np_(Wtg[taus][:, Si][:, :, Si])
    e_t = rel(got_t, Wt_ref)
    print(f"[{cfg.name}] screen NI={NI}: W(i nu) rel {e_w:.2e}, W(tau) rel {e_t:.2e}")
    assert e_w < 1e-10 and e_t < 1e-10


@pytest.mark.parametrize("ni", [400, 512, 513, 1024])
def test_screen_panel_sizes(torch, ni):
    """The FP64 screen at C2's product-basis size (400), at a multiple of the 64-column outer panel
    (512), one past it (513, a last panel of one column) and at the largest NI (1024), against the
    oracle on sampled frequencies of a synthetic negative-definite P(i nu) with a non-Hermitian part."""
    import paper_1602_02313_amd as amd
    cfg = gi.C2.replace(ni=ni, name=f"c2_ni{ni}")
    prob = gi.make_problem(cfg)
    run = amd.GWRun(cfg.nk, prob.kmq, prob.nb, prob.ni, prob.tau, cfg.beta, cfg.niw_f, cfg.niw_b,
                    cfg.scale, prob.eps, prob.v, prob.n_target, precision=amd.FP64, q_batch=1)
    q, niw = 2, cfg.niw_b
    rng = np.random.default_rng(ni)
    d = 1.0 / (1.0 + np.arange(ni) / 16.0)
    B = (rng.normal(size=(ni, ni)) + 1j * rng.normal(size=(ni, ni))) * np.sqrt(d)[:, None]
    P0 = -(B @ B.conj().T) / ni * 0.02
    C = rng.normal(size=(ni, ni)) + 1j * rng.normal(size=(ni, ni))
    P1 = (C - C.T) * 1e-3                                # a non-Hermitian part as well
    nu = o.matsubara(o.BOSON, niw, cfg.beta)
    lor = 1.0 / (1.0 + (nu / 0.5) ** 2)
    Piw = lor[:, None, None] * P0[None] + (lor ** 2)[:, None, None] * P1[None]
    run.P_iw[:Piw.size].copy_(torch.from_numpy(Piw.ravel()))
    vq = torch.from_numpy(np.asarray(prob.v[q], dtype=np.float64)).to("cuda")
    run.ctx.screen(q, 1, run.P_iw, vq, run.Wt_iw, run.R_iw, run.info)
    torch.cuda.synchronize()
    assert int(run.info[:niw].abs().max()) == 0
    nus = [0, 1, niw // 2, niw - 1]
    W, R = o.screen(Piw[nus], prob.v[q])
    Wg = np_(run.Wt_iw[:Piw.size].view(niw, ni, ni)[nus])
    Rg = np_(run.R_iw[:Piw.size].view(niw, ni, ni)[nus])
    e_w, e_r = rel(Wg, W), rel(Rg, R)
    print(f"screen NI={ni}: W(i nu) rel {e_w:.2e}, R rel {e_r:.2e}")
    assert e_w < 1e-10 and e_r < 1e-10
