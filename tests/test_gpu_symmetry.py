"""The tau mirror P(q, tau) = P(q, beta - tau) of the split-BF16 pair-space polarization.

With inputs that have the time-reversal symmetry (the symmetric generator), computing the points
i <= (N - 1) / 2 and copying the others reproduces the full computation and the oracle; with
inputs that lack it, the copied points are wrong, which is why it is the caller's assertion.
"""
import numpy as np
import pytest

import gwinputs as gi
import oracle as o
from gpu_util import make_run, np_, rel
from test_gpu_mixed import LONGTAU
from test_gpu_parity import SMALL, UNEVEN, oracle_G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _both(torch, cfg, q, symmetric):
    import paper_1602_02313_amd as amd
    prob, run = make_run(cfg, precision=amd.BF16X3)
    M = torch.empty(int(run.mpre[q + 1] - run.mpre[q]), dtype=torch.complex64, device="cuda")
    run.ctx.synth_M(cfg.seed, q, 1, int(symmetric), amd.C64, M)
    run.green0(0.0)
    NI, ntau = int(prob.ni[q]), prob.tau.size
    n = ntau * NI * NI
    run.ctx.polarization(q, 1, M, amd.C64, run.G_tau, amd.BF16X3, run.P_tau)
    full = np_(run.P_tau[:n]).reshape(ntau, NI, NI).copy()
    run.ctx.set_tau_mirror(True)
    run.P_tau.fill_(float("nan"))
    run.ctx.polarization(q, 1, M, amd.C64, run.G_tau, amd.BF16X3, run.P_tau)
    run.ctx.set_tau_mirror(False)
    mir = np_(run.P_tau[:n]).reshape(ntau, NI, NI)
    return prob, full, mir


@pytest.mark.parametrize("cfg,q", [(SMALL, 1), (UNEVEN, 2), (LONGTAU, 1)])
def test_tau_mirror_matches_full_and_oracle(torch, cfg, q):
    prob, full, mir = _both(torch, cfg, q, True)
    ntau = prob.tau.size
    assert np.all(np.isfinite(mir))
    # the computed half is the same work; the copied half equals the full computation to rounding
    h = (ntau + 1) // 2
    assert np.array_equal(mir[:h], full[:h])
    e_full = rel(mir, full)
    ref = o.polarization(gi.MGenerator(cfg).q_blocks(q), oracle_G(prob), prob.kmq[q], cfg.scale)
    e_ref = rel(mir, ref)
    print(f"{cfg.name} q={q}: mirror vs full {e_full:.2e}, vs oracle {e_ref:.2e}")
    assert e_full < 1e-6 and e_ref < 1e-5


def test_tau_mirror_needs_the_symmetry(torch):
    prob, full, mir = _both(torch, SMALL, 1, False)
    e = rel(mir, full)
    print(f"non-symmetric inputs: mirror vs full {e:.2e}")
    assert e > 1e-2
