"""GPU parity of the screen's two paths in one call: the blocked Hermitian sweep (P(i nu) Hermitian, A =
1 - v^1/2 P v^1/2 positive definite) and the pivoting Gauss-Jordan (P not Hermitian, or A indefinite,
whose sweep meets a non-positive pivot and is redone with pivoting), against the oracle's screen at
rel 1e-10.

Frequencies of one call: 0, 4: P negative definite (the sweep); 1: P positive with A indefinite (the
sweep fails, the matrix is rebuilt and eliminated with pivoting); 2: a non-Hermitian P (pivoting
elimination); 3: a Hermitian P with an anti-Hermitian part of 1e-9 of its largest element (below the
1e-6 tolerance: the sweep inverts the Hermitian part, compared with the oracle on that part, while R
= W~ - v P v keeps the P given); the
others negative definite at other scales.  NI = 64 (one block), 150 (two blocks and a ragged one) and
200.
"""
import numpy as np
import pytest

import gwinputs as gi
import oracle as o
from gpu_util import make_run, np_, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _inputs(ni, niw, seed):
    rng = np.random.default_rng(seed)
    B = (rng.normal(size=(ni, ni)) + 1j * rng.normal(size=(ni, ni))) / np.sqrt(ni)
    C = rng.normal(size=(ni, ni)) + 1j * rng.normal(size=(ni, ni))
    H = B @ B.conj().T
    P = np.empty((niw, ni, ni), dtype=complex)
    for n in range(niw):
        P[n] = -H * 0.02 / (1.0 + n)
    P[1] = H * 0.05                                    # A indefinite
    P[2] = -H * 0.02 + (C - C.T) * 1e-3                # not Hermitian
    anti = (C - C.conj().T) / 2.0
    P[3] = -H * 0.02 + anti * (1e-9 * np.abs(H * 0.02).max() / np.abs(anti).max())
    return P


@pytest.mark.parametrize("ni", [64, 150, 200])
def test_screen_hermitian_and_pivoting_paths(torch, ni):
    cfg = gi.tiny(name=f"hs{ni}", grid=(2, 1, 1), nocc=2, nemp=2, ni=ni, ntau=8, beta=10.0, niw=8)
    prob, run = make_run(cfg, q_batch=1)
    niw = cfg.niw_b
    P = _inputs(ni, niw, ni)
    v = prob.v[0]
    run.P_iw[:P.size].copy_(torch.from_numpy(P.ravel()))
    vq = torch.from_numpy(np.asarray(v, dtype=np.float64)).to("cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    run.ctx.screen(0, 1, run.P_iw, vq, run.Wt_iw, run.R_iw, run.info, flags)
    torch.cuda.synchronize()
    assert int(run.info[:niw].abs().max()) == 0 and int(flags.item()) == 0
    Wg = np_(run.Wt_iw[:P.size]).reshape(P.shape)
    Rg = np_(run.R_iw[:P.size]).reshape(P.shape)
    Pref = P.copy()
    Pref[3] = 0.5 * (P[3] + P[3].conj().T)            # the Hermitian part is what the sweep inverts
    W, _ = o.screen(Pref, v)
    R = W - v[None, :, None] * P * v[None, None, :]  # R = W~ - v P v with the P given
    for n in range(niw):
        ew, er = rel(Wg[n], W[n]), rel(Rg[n], R[n])
        print(f"NI={ni} nu={n}: W rel {ew:.2e}, R rel {er:.2e}")
        assert ew < TOL and er < TOL, (n, ew, er)
    # the Hermitian results are Hermitian to rounding
    for n in (0, 3, 4):
        assert np.abs(Wg[n] - Wg[n].conj().T).max() <= 1e-12 * np.abs(Wg[n]).max()
    # the near-Hermitian frequency against the exact inverse of its own P: the anti-Hermitian part
    # (1e-9 of P) is what the sweep leaves out
    W3, _ = o.screen(P[3:4], v)
    assert rel(Wg[3], W3[0]) < 1e-7
