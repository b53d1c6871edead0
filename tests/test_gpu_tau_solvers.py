"""GPU parity of the paper's tau-domain solvers (msgw_wt_tau_system, msgw_dyson_tau) against the
oracle's wt_tau_system and dyson_tau, FP64 gate rel 1e-10, and their agreement with the
Matsubara-axis path to discretisation error.

Shapes: the W~ system at orders ntau * NI = 777, 1470 and 2520 (one per register layout of the
Gauss-Jordan panel), two q per call with unequal NI, and at 1024 and 1040 (the largest order of the
two-level elimination and the first of the one-level one); the Dyson solve on a UPM mesh of 31 points
whose dense grid has 41 nodes, with uneven band counts.
"""
import numpy as np
import pytest

import gwinputs as gi
import oracle as o
from gpu_util import make_run, np_, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10

WSYS = {
    "n777": gi.tiny(name="ws777", grid=(2, 1, 1), nocc=3, nemp=3, ni=37, ntau=20, beta=12.0, niw=16, mesh="upm"),
    "n1470": gi.Config(name="ws1470", grid=(3, 1, 1), bands=((2, -1.0, -0.2), (4, 0.1, 1.5)), nb=None, ni=None,
                       nb_range=(3, 6), ni_range=(40, 70), ntau=20, mesh="upm", beta=20.0, niw_f=16, niw_b=16),
    "n2520": gi.tiny(name="ws2520", grid=(2, 1, 1), nocc=2, nemp=3, ni=120, ntau=20, beta=10.0, niw=16),
    # the largest order of the two-level elimination and the first of the one-level one
    "n1024": gi.tiny(name="ws1024", grid=(2, 1, 1), nocc=3, nemp=3, ni=64, ntau=15, beta=10.0, niw=16),
    "n1040": gi.tiny(name="ws1040", grid=(2, 1, 1), nocc=3, nemp=3, ni=65, ntau=15, beta=10.0, niw=16),
}
DYS = gi.Config(name="dys", grid=(3, 1, 1), bands=((3, -1.0, -0.2), (4, 0.1, 1.5)), nb=None, ni=6,
                nb_range=(4, 7), ntau=30, mesh="upm", beta=20.0, niw_f=64, niw_b=16)


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _oracle_P(prob, cfg, q):
    g = gi.MGenerator(cfg)
    G = o.green0(prob.eps, prob.nb, prob.tau, cfg.beta)
    return o.polarization(g.q_blocks(q), G, prob.kmq[q], cfg.scale)


@pytest.mark.parametrize("name", list(WSYS))
def test_wt_tau_system_matches_oracle(torch, name):
    import paper_1602_02313_amd as amd
    cfg = WSYS[name]
    prob, run = make_run(cfg)
    qs = [0, 1]
    nt = prob.tau.size
    print(f"\n[{name}] W~ tau system, q = {qs}, orders {[nt * int(prob.ni[q]) for q in qs]}", flush=True)
    P = [_oracle_P(prob, cfg, q) for q in qs]
    v = [prob.v[q][: int(prob.ni[q])] for q in qs]
    Pd = torch.from_numpy(np.concatenate([p.ravel() for p in P])).to("cuda")
    vd = torch.from_numpy(np.concatenate(v)).to("cuda")
    W = torch.zeros_like(Pd)
    info = torch.full((len(qs),), -7, dtype=torch.int32, device="cuda")
    nbytes = run.ctx.tau_solver_work_size(amd.TS_WTILDE, qs[0], len(qs))
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    run.ctx.wt_tau_system(qs[0], len(qs), Pd, vd, W, info, work, nbytes)
    torch.cuda.synchronize()
    assert np_(info).tolist() == [0, 0]
    got = np_(W)
    off = 0
    for q, p, vq in zip(qs, P, v):
        ref = o.wt_tau_system(p, vq, prob.tau, cfg.beta)
        g = got[off: off + ref.size].reshape(ref.shape)
        off += ref.size
        e = rel(g, ref)
        print(f"q={q}: rel {e:.2e}")
        assert e < TOL, (q, e)


def test_wt_tau_system_agrees_with_screen_route(torch):
    """On one q the library's tau system and its nu-axis chain (polarization, P(tau) -> P(i nu), screen,
    W~(tau)) differ by the discretisation error of the two routes, the same difference the oracle's two
    routes show on these inputs (the oracle pins the convergence rates)."""
    import paper_1602_02313_amd as amd
    cfg = WSYS["n777"]
    prob, run = make_run(cfg)
    q = 0
    NI, nt = int(prob.ni[q]), prob.tau.size
    g = gi.MGenerator(cfg)
    M = torch.from_numpy(g.q_packed(q)).to("cuda")
    run.green0(0.0)
    run.sig_tau.zero_()
    run.sig_x.zero_()
    run.q_block(lambda r, q0, nq: M, q, 1)
    Pd = run.P_tau[: nt * NI * NI].clone()
    vd = run.v[int(run.vpre[q]): int(run.vpre[q]) + NI].clone()
    W = torch.zeros_like(Pd)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    nbytes = run.ctx.tau_solver_work_size(amd.TS_WTILDE, q, 1)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    run.ctx.wt_tau_system(q, 1, Pd, vd, W, info, work, nbytes)
    torch.cuda.synchronize()
    got_tau = np_(W).reshape(nt, NI, NI)
    got_nu = np_(run.Wt_tau[: nt * NI * NI]).reshape(nt, NI, NI)
    # the oracle's two routes on the same P
    P = _oracle_P(prob, cfg, q)
    v = prob.v[q][:NI]
    ref_tau = o.wt_tau_system(P, v, prob.tau, cfg.beta)
    ref_nu = o.wt_tau(o.screen(o.tau_to_iw(P, prob.tau, cfg.beta, o.BOSON, cfg.niw_b), v)[1], P, v,
                      prob.tau, cfg.beta)
    scale = np.abs(ref_nu).max()
    d_gpu = np.abs(got_tau - got_nu).max() / scale
    d_ref = np.abs(ref_tau - ref_nu).max() / scale
    print(f"tau system vs nu route: GPU {d_gpu:.3e}, oracle {d_ref:.3e} (max |diff| / max |W~|)")
    assert abs(d_gpu - d_ref) < 1e-8
    assert rel(got_tau, ref_tau) < TOL and rel(got_nu, ref_nu) < TOL


def _dyson_inputs(prob, cfg, seed=7):
    """Sigma^c(tau) of two fermionic poles per state (weights in [0.01, 0.05], poles in [-1, 1]) and a
    static self-energy in [-0.1, 0.1], zero on the padded bands."""
    rng = np.random.default_rng(seed)
    nk, nbmax, nt = cfg.nk, prob.eps.shape[1], prob.tau.size
    sig = np.zeros((nk, nbmax, nt))
    sst = np.zeros((nk, nbmax))
    for k in range(nk):
        for n in range(int(prob.nb[k])):
            for _ in range(2):
                sig[k, n] += rng.uniform(0.01, 0.05) * o.green0_tau(rng.uniform(-1.0, 1.0), prob.tau, cfg.beta)
            sst[k, n] = rng.uniform(-0.1, 0.1)
    return sig, sst


def test_dyson_tau_matches_oracle_and_the_matsubara_route(torch):
    import paper_1602_02313_amd as amd
    cfg = DYS
    prob, run = make_run(cfg)
    nk, nbmax, nt, beta = cfg.nk, prob.eps.shape[1], prob.tau.size, cfg.beta
    sig, sst = _dyson_inputs(prob, cfg)
    mu = 0.05
    print(f"\n[dys] tau Dyson, {nk} k, bands {list(prob.nb)}, dense grid {o.dense_grid(prob.tau, beta).size}",
          flush=True)
    # the Matsubara route through the library at the same fixed mu
    run.sig_tau.copy_(torch.from_numpy(sig))
    run.sig_x.copy_(torch.from_numpy(sst))
    run.mu.fill_(mu)
    run.sigma_to_iw()
    run._dyson(search=False)
    G_nu = np_(run.G_tau).copy()
    # the tau route on k = 1, 2 (k = 0 must stay untouched)
    k0, nkc = 1, nk - 1
    Gt = torch.zeros((nk, nbmax, nt), dtype=torch.float64, device="cuda")
    info = torch.full((nkc * nbmax,), -7, dtype=torch.int32, device="cuda")
    nbytes = run.ctx.tau_solver_work_size(amd.TS_DYSON, k0, nkc)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    run.ctx.dyson_tau(k0, nkc, run.eps, run.sig_x, run.mu, run.sig_tau, Gt, info, work, nbytes)
    torch.cuda.synchronize()
    assert (np_(info) == 0).all()
    got = np_(Gt)
    assert (got[0] == 0).all()
    # the oracle's two routes
    sig_iw = np.moveaxis(o.tau_to_iw(np.moveaxis(sig, -1, 0), prob.tau, beta, o.FERMION, cfg.niw_f), 0, -1)
    ref_nu = o.dyson(prob.eps, prob.nb, sst, sig_iw, beta, prob.tau, prob.n_target, mu0=mu, search=False)["G_tau"]
    worst, d_gpu, d_ref = 0.0, 0.0, 0.0
    for k in range(k0, k0 + nkc):
        for n in range(int(prob.nb[k])):
            _, _, ref = o.dyson_tau(prob.eps[k, n] - mu, sst[k, n], sig[k, n], prob.tau, beta)
            worst = max(worst, np.abs(got[k, n] - ref).max() / np.abs(ref).max())
            d_gpu = max(d_gpu, np.abs(got[k, n] - G_nu[k, n]).max())
            d_ref = max(d_ref, np.abs(ref - ref_nu[k, n]).max())
        assert (got[k, int(prob.nb[k]):] == 0).all()
    print(f"tau Dyson vs oracle: max rel {worst:.2e}; tau vs i w route: GPU {d_gpu:.3e}, oracle {d_ref:.3e}")
    assert worst < TOL
    assert abs(d_gpu - d_ref) < 1e-9
    assert d_gpu < 1e-2


def test_tau_solvers_refuse_unsupported_shapes(torch):
    import paper_1602_02313_amd as amd
    cfg = gi.tiny(name="big", grid=(2, 1, 1), nocc=2, nemp=2, ni=200, ntau=20, beta=10.0, niw=8)
    prob, run = make_run(cfg)
    with pytest.raises(amd.MsgwError) as e:
        run.ctx.tau_solver_work_size(amd.TS_WTILDE, 0, 1)
    assert e.value.code == amd.ENOTSUP
    # a mesh whose points are not multiples of tau_1 - tau_0 has no dense grid
    cfg2 = gi.tiny(name="odd", grid=(2, 1, 1), nocc=2, nemp=2, ni=4, ntau=20, beta=10.0, niw=8)
    prob2 = gi.make_problem(cfg2)
    tau = prob2.tau.copy()
    tau[1] *= 0.7
    tau[-2] = cfg2.beta - tau[1]
    run2 = amd.GWRun(cfg2.nk, prob2.kmq, prob2.nb, prob2.ni, tau, cfg2.beta, cfg2.niw_f, cfg2.niw_b, cfg2.scale,
                     prob2.eps, prob2.v, prob2.n_target)
    with pytest.raises(amd.MsgwError) as e:
        run2.ctx.tau_solver_work_size(amd.TS_DYSON, 0, 1)
    assert e.value.code == amd.ESHAPE
