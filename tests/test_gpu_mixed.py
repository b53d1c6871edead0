"""GPU parity of the mixed-precision contractions (FP32, split BF16 and split FP16) against the FP64 oracle.

Gates (relative Frobenius error per array against the FP64 oracle; the split-precision tolerance of
the path is rel 1e-6 on Sigma):
  FP32 MFMA:          P and Sigma^c <= 2e-6 (the plain FP32 path: 4-deep MFMA steps round the
                      FP32 accumulators about four times as often as the split paths)
  F16X3 (split FP16): P and Sigma^c <= 1e-6, on every shape
  BF16X3 (split BF16) P and Sigma^c <= 1e-5 on the small shapes: its 8-bit significand leaves
                      ~2^-16 per product, which short sums do not average below 1e-6 (measured
                      0.9-3.1e-6); Sigma^c <= 1e-6 at the full shapes
Beside the Frobenius norm each comparison bounds the worst tau slice (relative to that slice) and
the largest absolute error (relative to the largest entry), at SLICE x the gate.
The inputs M are stored in complex64 for these paths; that rounding (2^-24 relative) is part
of the measured error.
"""
import numpy as np
import pytest

import gwinputs as gi
import oracle as o
from gpu_util import check, make_run, np_, rel
from test_gpu_parity import SMALL, TILES, UNEVEN, _oracle_pw, oracle_G

pytestmark = pytest.mark.gpu

GATE = {1: 2e-6, 2: 1e-5, 3: 1e-6}
FULL_GATE = 1e-6      # Sigma^c of every precision at the full shapes
PRECS = (1, 2, 3)
# more than 96 tau points: the pair-space polarization runs its tau axis in chunks of 96
LONGTAU = gi.tiny(name="longtau", grid=(2, 1, 1), nocc=3, nemp=3, ni=41, ntau=120, beta=30.0, niw=16)


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _variants(prec, op):
    """Indices of the compiled tile variants (just [0] when the library is not built)."""
    try:
        import paper_1602_02313_amd as amd
        return list(range(amd.load_library().msgw_variant_count(op, prec)))
    except ImportError:
        return [0]


def _m64(cfg, run, g):
    import torch
    flat = np.concatenate([g.q_packed(q) for q in range(cfg.nk)]).astype(np.complex64)
    return torch.from_numpy(flat).to(run.device)


def _small_cases(op):
    return [(p, v) for p in PRECS for v in _variants(p, op)]


@pytest.mark.parametrize("prec,variant", _small_cases(0))
@pytest.mark.parametrize("cfg", [SMALL, UNEVEN, TILES, LONGTAU])
def test_polarization_mixed(torch, cfg, prec, variant):
    import paper_1602_02313_amd as amd
    prob, run = make_run(cfg, precision=prec, q_batch=cfg.nk)
    g = gi.MGenerator(cfg)
    M = _m64(cfg, run, g)
    run.green0(0.0)
    run.ctx.set_variant(0, prec, variant)
    run.ctx.polarization(0, cfg.nk, M, amd.C64, run.G_tau, prec, run.P_tau)
    torch.cuda.synchronize()
    G = oracle_G(prob)
    P = np_(run.P_tau)
    for q in range(cfg.nk):
        ref = o.polarization(g.q_blocks(q), G, prob.kmq[q], cfg.scale)
        got = P[run.ppre[q]:run.ppre[q + 1]].reshape(ref.shape)
        check(f"P {cfg.name} q={q} prec={prec} variant={variant}", got, ref, GATE[prec], 0)


@pytest.mark.parametrize("prec,variant", _small_cases(1))
@pytest.mark.parametrize("cfg", [SMALL, UNEVEN, TILES, LONGTAU])
def test_self_energy_mixed(torch, cfg, prec, variant):
    import paper_1602_02313_amd as amd
    prob, run = make_run(cfg, precision=prec, q_batch=1)
    g = gi.MGenerator(cfg)
    G = oracle_G(prob)
    run.green0(0.0)
    run.sig_tau.zero_()
    run.ctx.set_variant(1, prec, variant)
    ref = 0
    off = np.concatenate([[0], np.cumsum([g.q_packed(q).size for q in range(cfg.nk)])])
    M = _m64(cfg, run, g)
    for q in range(cfg.nk):
        _, _, _, _, Wt = _oracle_pw(prob, g, q, G)
        run.Wt_tau[:Wt.size].copy_(torch.from_numpy(Wt.ravel()))
        run.ctx.self_energy(q, 1, M[off[q]:off[q + 1]], amd.C64, run.G_tau, run.Wt_tau, prec, run.sig_tau)
        ref = ref + o.sigma_c(g.q_blocks(q), G, prob.kmq[q], Wt, cfg.scale)
    torch.cuda.synchronize()
    check(f"Sigma {cfg.name} prec={prec} variant={variant}", np_(run.sig_tau), ref, GATE[prec], -1)


@pytest.mark.parametrize("prec", PRECS)
def test_end_to_end_c1_mixed(torch, prec):
    import paper_1602_02313_amd as amd
    cfg = gi.C1
    prob = gi.make_problem(cfg)
    g = gi.MGenerator(cfg)
    hist = o.run_loop(prob, g, "g0w0", 1)
    _, run = make_run(cfg, precision=prec, q_batch=8)
    src = amd.HostM(lambda q: g.q_packed(q), amd.C64)
    out = run.run(src, "g0w0", 1)
    torch.cuda.synchronize()
    ex = rel(np_(run.sig_x), hist[0]["sigx"])
    eg = abs(out[0]["gap"] - hist[0]["gap"])
    print(f"c1 G0W0 prec={prec}: Sigma^x rel {ex:.2e}, gap err {eg:.3e} Ha (gap {hist[0]['gap']:.4f} Ha)")
    check(f"c1 G0W0 Sigma^c prec={prec}", np_(run.sig_tau), hist[0]["sigc_tau"], GATE[prec], -1)
    assert ex < 1e-6


# ---------------------------------------------------------------------------------------------
# full-size shapes (64 k-points, 64 bands, NI = 400, 81 tau points), sampled against the oracle
# ---------------------------------------------------------------------------------------------
C2 = gi.C2


@pytest.fixture(scope="module")
def c2_setup(torch):
    import paper_1602_02313_amd as amd
    prob = gi.make_problem(C2)
    run = amd.GWRun(C2.nk, prob.kmq, prob.nb, prob.ni, prob.tau, C2.beta, C2.niw_f, C2.niw_b,
                    C2.scale, prob.eps, prob.v, prob.n_target, precision=amd.BF16X3, q_batch=1)
    size = int(run.mpre[1] - run.mpre[0])
    M = torch.empty(size, dtype=torch.complex64, device="cuda")
    run.ctx.synth_M(C2.seed, 0, 1, 1, amd.C64, M)
    run.green0(0.0)
    torch.cuda.synchronize()
    return prob, run, M


FULL_P = [(p, v) for p in PRECS for v in _variants(p, 0)]
FULL_S = [(p, v) for p in PRECS for v in _variants(p, 1)]


@pytest.mark.parametrize("prec,variant", FULL_P)
def test_full_size_polarization_sampled(torch, c2_setup, prec, variant):
    import paper_1602_02313_amd as amd
    prob, run, M = c2_setup
    run.ctx.set_variant(0, prec, variant)
    run.ctx.polarization(0, 1, M, amd.C64, run.G_tau, prec, run.P_tau)
    run.ctx.set_variant(0, prec, 0)
    torch.cuda.synchronize()
    NI, ntau = 400, prob.tau.size
    P = np_(run.P_tau[:ntau * NI * NI]).reshape(ntau, NI, NI)
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(NI, 12, replace=False))
    cols = np.sort(np.concatenate([rows[:4], rng.choice(NI, 8, replace=False)]))
    taus = [0, 17, 40, 80]
    g = gi.MGenerator(C2)
    sel = np.union1d(rows, cols)
    blocks = [g.block(0, k, rows=sel) for k in range(C2.nk)]
    G = oracle_G(prob)
    ri, ci = np.searchsorted(sel, rows), np.searchsorted(sel, cols)
    ref = o.polarization(blocks, G, prob.kmq[0], C2.scale, taus=taus, rows=ri, cols=ci)
    got = P[np.ix_(taus, rows, cols)]
    check(f"full-size P prec={prec} variant={variant} ({got.size} sampled entries)", got, ref, GATE[prec], 0)


@pytest.mark.parametrize("prec,variant", FULL_S)
def test_full_size_self_energy_sampled(torch, c2_setup, prec, variant):
    import paper_1602_02313_amd as amd
    prob, run, M = c2_setup
    NI, ntau = 400, prob.tau.size
    rng = np.random.default_rng(1)
    # a Hermitian W~(tau) with the magnitude profile of the screened interaction (decaying in I)
    d = 1.0 / (1.0 + np.arange(NI) / 16.0)
    W = (rng.normal(size=(ntau, NI, NI)) + 1j * rng.normal(size=(ntau, NI, NI))) * 0.01
    W = W + np.conj(np.swapaxes(W, 1, 2)) + np.diag(d)[None] * 5.0
    W = W * np.sqrt(d)[None, :, None] * np.sqrt(d)[None, None, :]
    run.Wt_tau[:W.size].copy_(torch.from_numpy(W.ravel()))
    run.sig_tau.zero_()
    run.ctx.set_variant(1, prec, variant)
    run.ctx.self_energy(0, 1, M, amd.C64, run.G_tau, run.Wt_tau, prec, run.sig_tau)
    run.ctx.set_variant(1, prec, 0)
    torch.cuda.synchronize()
    S = np_(run.sig_tau)
    g = gi.MGenerator(C2)
    G = oracle_G(prob)
    ks, taus = [0, 37], [0, 40, 80]
    Mq = [g.block(0, k) if k in ks else None for k in range(C2.nk)]
    ref = o.sigma_c(Mq, G, prob.kmq[0], W, C2.scale, taus=taus, ks=ks)
    got = S[np.ix_(ks, np.arange(S.shape[1]), taus)]
    check(f"full-size Sigma prec={prec} variant={variant}", got, ref, FULL_GATE, -1)


# ---------------------------------------------------------------------------------------------
# physical scale: with Omega = N_occ * sum_I v_I / (1 + I/16) (about 3.5e3 for C1) the exchange
# self-energy is O(1 Ha), as in a real solid, and the gap proxy is a few mHa; the split paths must
# then reproduce the oracle's gap within 1 meV, in G0W0 and along a self-consistent loop
# ---------------------------------------------------------------------------------------------
MEV = 1e-3 / 27.211386245988
C1_PHYS = gi.C1.replace(omega=3528.0, name="c1_physical_scale")


@pytest.fixture(scope="module")
def c1_phys_oracle():
    prob = gi.make_problem(C1_PHYS)
    g = gi.MGenerator(C1_PHYS)
    return prob, g, o.run_loop(prob, g, "g0w0", 1), o.run_loop(prob, g, "scgw", 3)


@pytest.mark.parametrize("prec", PRECS)
def test_gap_physical_scale(torch, c1_phys_oracle, prec):
    import paper_1602_02313_amd as amd
    prob, g, h0, hsc = c1_phys_oracle
    _, run = make_run(C1_PHYS, precision=prec, q_batch=8)
    src = amd.HostM(lambda q: g.q_packed(q), amd.C64)
    out0 = run.run(src, "g0w0", 1)
    torch.cuda.synchronize()
    es = check(f"physical scale Sigma^c prec={prec}", np_(run.sig_tau), h0[0]["sigc_tau"], GATE[prec], -1)
    e0 = abs(out0[0]["gap"] - h0[0]["gap"])
    outs = run.run(src, "scgw", 3)
    esc = [abs(a["gap"] - b["gap"]) for a, b in zip(outs, hsc)]
    print(f"physical scale prec={prec}: Sigma^c rel {es:.2e}; G0W0 gap {h0[0]['gap'] * 1e3:.4f} mHa, "
          f"err {e0 / MEV:.2e} meV; scGW gap errors (meV) {[f'{x / MEV:.2e}' for x in esc]}")
    assert e0 < MEV and max(esc) < MEV


# ---------------------------------------------------------------------------------------------
# the scGW iteration as a HIP graph: every replay must reproduce the eager iteration and follow
# the oracle's self-consistent loop (FP64: 1e-10; split: the gap within 1 meV)
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("prec", [0, 2, 3])
def test_graph_replays_match_eager(torch, c1_phys_oracle, prec):
    import paper_1602_02313_amd as amd
    cfg = C1_PHYS
    prob = gi.make_problem(cfg)
    hsc = c1_phys_oracle[3]
    _, run = make_run(cfg, precision=prec, q_batch=4)
    mdt = amd.C128 if prec == 0 else amd.C64
    ct = torch.complex128 if prec == 0 else torch.complex64
    M = torch.empty(int(run.mpre[-1]), dtype=ct, device="cuda")
    run.ctx.synth_M(cfg.seed, 0, cfg.nk, 1, mdt, M)
    src = amd.ResidentM(M, run.mpre)
    niter = 3
    eager, eager_G = [], []
    run.green0(0.0)
    run.mu.zero_()
    for _ in range(niter):
        run.iteration(src)
        eager.append(run._record())
        eager_G.append(np_(run.G_tau).copy())
    run.green0(0.0)
    run.mu.zero_()
    g = run.capture_iteration(src)
    for it in range(niter):
        # eager work and a synchronization between replays
        junk = torch.ones(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        g.replay()
        rec = run._record()
        eg = rel(np_(run.G_tau), eager_G[it])
        print(f"graph prec={prec} replay {it}: gap {rec['gap']:.9f} (eager {eager[it]['gap']:.9f}), "
              f"G rel {eg:.2e}, flags {rec['flags']}")
        assert rec["flags"] == eager[it]["flags"] == 0
        assert abs(rec["gap"] - eager[it]["gap"]) < 1e-9 and abs(rec["N"] - eager[it]["N"]) < 1e-9
        assert eg < 1e-10
        # against the oracle's scGW iteration it
        eo = rel(np_(run.G_tau), hsc[it]["G_tau"])
        go = abs(rec["gap"] - hsc[it]["gap"])
        print(f"   vs oracle: G rel {eo:.2e}, gap err {go / MEV:.2e} meV")
        if prec == 0:
            assert eo < 1e-10 and go < 1e-10
        else:
            assert go < MEV
        del junk


# ---------------------------------------------------------------------------------------------
# the whole chain P -> P(i nu) -> W~(i nu) -> W~(tau) -> Sigma^c at the block shapes of the
# 64-band, NI = 400 workload (81-point power mesh, beta = 200, 128 Matsubara points) on a 2^3
# k-grid, so that the oracle computes every step of one q in seconds; Sigma^c is compared on
# all bands of two k points at every tau
# ---------------------------------------------------------------------------------------------
C2_BLOCKS = gi.C2.replace(grid=(2, 2, 2), name="c2_blocks_k8")


@pytest.fixture(scope="module")
def c2_chain_oracle():
    prob = gi.make_problem(C2_BLOCKS)
    g = gi.MGenerator(C2_BLOCKS)
    G = oracle_G(prob)
    q = 1
    Mq = g.q_blocks(q)
    P, Piw, Wiw, R, Wt = _oracle_pw(prob, g, q, G)
    ks = [0, 5]
    sig = o.sigma_c(Mq, G, prob.kmq[q], Wt, C2_BLOCKS.scale, ks=ks)
    return prob, g, q, ks, P, Wt, sig


@pytest.mark.parametrize("prec", PRECS)
def test_chain_c2_blocks(torch, c2_chain_oracle, prec):
    import paper_1602_02313_amd as amd
    prob, g, q, ks, Pref, Wref, Sref = c2_chain_oracle
    cfg = C2_BLOCKS
    _, run = make_run(cfg, precision=prec, q_batch=1)
    M = torch.from_numpy(g.q_packed(q).astype(np.complex64)).to(run.device)
    run.green0(0.0)
    run.sig_tau.zero_()
    run.sig_x.zero_()
    run.q_block(lambda r, q0, nq: M, q, 1)
    torch.cuda.synchronize()
    NI, ntau = int(prob.ni[q]), prob.tau.size
    check(f"chain P prec={prec}", np_(run.P_tau[:ntau * NI * NI]).reshape(ntau, NI, NI), Pref, GATE[prec], 0)
    # the screen amplifies the error of P by its conditioning (|W~| / |v P v| ~ 5 at these scales)
    check(f"chain W~(tau) prec={prec}", np_(run.Wt_tau[:ntau * NI * NI]).reshape(ntau, NI, NI), Wref,
          10 * GATE[prec], 0, slices=False)
    # Sigma^c(tau) inherits the absolute error of W~(tau), so its slices near beta/2 are compared
    # on the scale of the whole array as well
    check(f"chain Sigma^c prec={prec}", np_(run.sig_tau)[ks], Sref, GATE[prec], -1, slices=False)
