"""msgw_dyson_noalloc, the Dyson entry point that allocates nothing (its scratch is a static device
array), against msgw_dyson through the C ABI: the same G(i w), G(tau), mu, N and flags on two calls
in a row, the second with a smaller problem (another context sharing the device's static array),
and the limit of that array refused on the host."""
import numpy as np
import pytest

import gwinputs as gi
import oracle as o
from gpu_util import make_run, np_, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10
LARGE = gi.C1.replace(grid=(3, 3, 2), name="noalloc_large")        # 18 k, 16 bands
SMALL = gi.tiny(name="noalloc_small", grid=(2, 1, 1), nocc=2, nemp=3, ni=5, ntau=12, beta=20.0, niw=16)


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _inputs(torch, cfg, prob, run, seed):
    """A static shift and a causal one-pole Sigma^c(i w) per state, seeded."""
    rng = np.random.default_rng(seed)
    nk, nb, niw = cfg.nk, run.nbmax, cfg.niw_f
    w = o.matsubara(o.FERMION, niw, cfg.beta)
    stat = rng.uniform(-0.05, 0.05, size=(nk, nb))
    amp = rng.uniform(0.05, 0.2, size=(nk, nb, 1))
    pole = rng.uniform(-0.5, 0.5, size=(nk, nb, 1))
    sig = amp / (1j * w[None, None, :] - pole)
    dev = run.device
    return (torch.from_numpy(stat).to(dev), torch.from_numpy(np.ascontiguousarray(sig)).to(dev), stat, sig)


def _call(torch, run, fn, stat_d, sig_d, n_target):
    dev = run.device
    mu = torch.zeros(1, dtype=torch.float64, device=dev)
    N = torch.zeros(1, dtype=torch.float64, device=dev)
    flags = torch.full((1,), -1, dtype=torch.int32, device=dev)
    G_iw = torch.empty_like(run.G_iw)
    G_tau = torch.empty_like(run.G_tau)
    fn(run.eps, stat_d, sig_d, n_target, 1, mu, G_iw, G_tau, N, flags)  # MSGW_MU_SEARCH
    torch.cuda.synchronize()
    return dict(mu=float(mu.item()), N=float(N.item()), flags=int(flags.item()), G_iw=np_(G_iw),
                G_tau=np_(G_tau))


def test_dyson_noalloc_matches_dyson(torch):
    # two calls in a row on the device's one static array: a larger problem, then a smaller one
    for seed, cfg in enumerate((LARGE, SMALL)):
        prob, run = make_run(cfg)
        stat_d, sig_d, stat, sig = _inputs(torch, cfg, prob, run, seed)
        ref = _call(torch, run, run.ctx.dyson, stat_d, sig_d, prob.n_target)
        got = _call(torch, run, run.ctx.dyson_noalloc, stat_d, sig_d, prob.n_target)
        eg, ei = rel(got["G_tau"], ref["G_tau"]), rel(got["G_iw"], ref["G_iw"])
        print(f"{cfg.name}: G(tau) rel {eg:.2e}, G(i w) rel {ei:.2e}, mu {got['mu']:.15f} "
              f"({ref['mu']:.15f}), N {got['N']:.12f}, flags {got['flags']}")
        assert eg < TOL and ei < TOL
        assert abs(got["mu"] - ref["mu"]) <= TOL * max(1.0, abs(ref["mu"]))
        assert abs(got["N"] - ref["N"]) <= TOL * ref["N"]
        assert got["flags"] == ref["flags"] == 0
        # and both against the oracle's Dyson step
        mask = np.arange(run.nbmax)[None, :] < prob.nb[:, None]
        d = o.dyson(prob.eps, prob.nb, stat, np.where(mask[..., None], sig, 0.0), cfg.beta, prob.tau,
                    prob.n_target)
        assert rel(got["G_tau"], d["G_tau"]) < TOL


def test_dyson_noalloc_refuses_beyond_its_array(torch):
    """2048 k x 64 bands = 131072 states exceed the 1 MiB array: refused on the host, before anything
    else (no workspace is attached to this context, so nothing could have been enqueued)."""
    import paper_1602_02313_amd as amd
    nk, nb = 2048, 64
    kmq = (np.arange(nk)[None, :] - np.arange(nk)[:, None]) % nk      # a ring of k points
    tau = np.linspace(0.0, 10.0, 8)
    ctx = amd.Context(0)
    ctx.set_problem(nk, kmq, np.full(nk, nb), np.full(nk, 4), tau, 10.0, 4, 4, -1.0 / nk)
    x = torch.zeros(8, dtype=torch.float64, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(amd.MsgwError) as e:
        ctx.dyson_noalloc(x, x, x, 1.0, 1, x, x, x, x, flags)
    assert e.value.code == amd.ENOTSUP
