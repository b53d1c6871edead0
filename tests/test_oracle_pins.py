"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed forms,
library routines for textbook special cases, brute force on a real-space toy,
literal loops, and identities stated in the paper.
"""
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.interpolate import CubicSpline

import gwinputs as gi
import oracle as o
from toy_realspace import NK, Toy

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# inputs: Philox known answers, mesh, generator symmetry
# ---------------------------------------------------------------------------
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        c = [int(x, 16) for x in r[:4]]
        key = int(r[4], 16) | (int(r[5], 16) << 32)
        want = [int(x, 16) for x in r[6:10]]
        got = gi.philox4x32_10(*[np.uint32(v) for v in c], key)
        assert [int(g) for g in got] == want


def test_upm_point_count_matches_paper():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "upm_mesh_paper.txt"))
            if l.strip() and not l.startswith("#")]
    for n, m, npts in rows:
        t = gi.upm_mesh(1000.0, int(n), int(m))
        assert t.size == int(npts)


@pytest.mark.parametrize("cfg", [gi.C1, gi.C2, gi.C3, gi.C5])
def test_tau_mesh_mirror(cfg):
    t = gi.tau_mesh(cfg)
    assert t.size == cfg.ntau + 1
    assert t[0] == 0.0 and t[-1] == cfg.beta
    assert np.all(np.diff(t) > 0)
    assert np.max(np.abs(t + t[::-1] - cfg.beta)) <= 1e-12 * cfg.beta
    if cfg.mesh == "upm":
        h = np.diff(t)
        # densest at both ends, spacing doubles between power intervals
        assert h[0] == pytest.approx(h[-1]) and h[0] == pytest.approx(h.min())


def test_generator_symmetry_and_variance():
    cfg = gi.tiny(grid=(3, 2, 1), nocc=3, nemp=2, ni=40)
    g = gi.MGenerator(cfg)
    mk, kmq = gi.minus_table(cfg), gi.kmq_table(cfg)
    sub = kmq.T
    for q in range(cfg.nk):
        for k in range(cfg.nk):
            M = g.block(q, k)
            # a: (k,q,n,m) -> (q-k, q, m, n), equal
            Ma = g.block(q, int(sub[q, k]))
            assert np.array_equal(M, np.swapaxes(Ma, 1, 2))
            # b: (k,q,n,m) -> (-k,-q,n,m), conjugate
            Mb = g.block(int(mk[q]), int(mk[k]))
            assert np.array_equal(M, np.conj(Mb))
    allM = np.concatenate([g.q_packed(q).reshape(-1) for q in range(cfg.nk)])
    assert np.isfinite(allM).all()
    # E|M^I|^2 = 1/(1+I/16): check the I = 0 row mean over all blocks
    M0 = np.concatenate([g.block(q, k)[0].ravel() for q in range(cfg.nk) for k in range(cfg.nk)])
    assert np.mean(np.abs(M0) ** 2) == pytest.approx(1.0, rel=0.25)


def test_uneven_counts_mirrored():
    cfg = gi.C4
    nb, ni, mk = gi.band_counts(cfg), gi.basis_sizes(cfg), gi.minus_table(cfg)
    assert nb.min() >= 96 and nb.max() <= 160 and ni.min() >= 500 and ni.max() <= 900
    assert np.array_equal(nb, nb[mk]) and np.array_equal(ni, ni[mk])
    assert len(set(nb.tolist())) > 20


# ---------------------------------------------------------------------------
# G0 and the transforms
# ---------------------------------------------------------------------------
def test_green0_closed_form_and_limits():
    beta = 20.0
    tau = gi.upm_mesh(beta, 40)
    E = np.array([-1.3, -0.2, 0.0, 0.05, 0.9])
    G = o.green0_tau(E, tau, beta)
    nF = 1.0 / (np.exp(beta * E) + 1.0)
    # 1 - n_F(E) = n_F(-E) keeps the direct formula free of cancellation
    direct = -np.exp(-E[:, None] * tau[None, :]) / (np.exp(-beta * E[:, None]) + 1.0)
    assert np.max(np.abs(G - direct) / np.abs(direct)) < 1e-14
    assert np.max(np.abs(G[:, 0] + G[:, -1] + 1.0)) < 1e-15
    assert np.max(np.abs(-G[:, -1] - nF)) < 1e-15
    # no overflow for large |beta E|
    Gx = o.green0_tau(np.array([-3000.0, 3000.0]), gi.upm_mesh(400.0, 40), 400.0)
    assert np.isfinite(Gx).all() and Gx[0, -1] == -1.0 and Gx[1, 0] == -1.0


def test_spline_matches_library_not_a_knot():
    t = gi.upm_mesh(30.0, 40)
    rng = np.random.default_rng(1)
    f = rng.normal(size=t.size)
    a, b, c, d = o.spline_not_a_knot(t, f)
    ref = CubicSpline(t, f, bc_type="not-a-knot")
    xs = np.sort(rng.uniform(0, 30.0, 500))
    i = np.clip(np.searchsorted(t, xs, side="right") - 1, 0, t.size - 2)
    dt = xs - t[i]
    S = a[i] + b[i] * dt + c[i] * dt ** 2 + d[i] * dt ** 3
    assert np.max(np.abs(S - ref(xs))) < 1e-12


@pytest.mark.parametrize("stat", [o.FERMION, o.BOSON])
def test_transform_exact_on_cubics(stat):
    """Spline-Filon quadrature is exact for global cubics (not-a-knot reproduces them).

    The reference integral uses repeated integration by parts,
    int_0^beta e^{iwt} p(t) dt = sum_j (-1)^j [p^(j)(t) e^{iwt}]_0^beta / (iw)^(j+1),
    a different formula from the Filon recurrence.
    """
    beta = 7.0
    t = gi.upm_mesh(beta, 30)
    coef = np.array([0.3, -1.1, 0.45, -0.07])          # p(t) = sum c_j t^j
    f = sum(cj * t ** j for j, cj in enumerate(coef))
    F = o.tau_to_iw(f, t, beta, stat, 40)
    w = o.matsubara(stat, 40, beta)
    der = [coef]
    for _ in range(3):
        c = der[-1]
        der.append(np.array([c[j] * j for j in range(1, len(c))] + [0.0]))
    ref = np.zeros(40, dtype=complex)
    for n, wn in enumerate(w):
        if wn == 0.0:
            ref[n] = sum(cj * beta ** (j + 1) / (j + 1) for j, cj in enumerate(coef))
            continue
        acc = 0
        for j in range(4):
            pj = lambda x: sum(cc * x ** i for i, cc in enumerate(der[j]))
            acc += (-1) ** j * (pj(beta) * np.exp(1j * wn * beta) - pj(0.0)) / (1j * wn) ** (j + 1)
        ref[n] = acc
    assert np.max(np.abs(F - ref)) < 1e-11 * np.max(np.abs(ref))


def test_fermion_transform_of_G0_converges_h4():
    """G0(i w_n) = 1/(i w_n - eps) follows from G0(tau) and eq. trans.
    With a reference energy different from eps the spline sees a smooth
    remainder and the error must fall as h^4."""
    beta = 10.0
    eps = np.array([-0.6, 0.35])
    errs = []
    for n in (20, 40, 80):
        t = np.linspace(0, beta, n + 1)
        G = o.green0_tau(eps, t, beta).T               # [ntau, 2]
        F = o.tau_to_iw(G, t, beta, o.FERMION, 16, e_ref=eps + 0.4)
        w = o.matsubara(o.FERMION, 16, beta)
        exact = 1.0 / (1j * w[:, None] - eps[None, :])
        errs.append(np.max(np.abs(F - exact)))
    assert errs[-1] < 1e-6
    assert errs[0] / errs[1] > 10 and errs[1] / errs[2] > 12
    # with the exact reference the result is exact
    t = gi.upm_mesh(beta, 20)
    G = o.green0_tau(eps, t, beta).T
    F = o.tau_to_iw(G, t, beta, o.FERMION, 16, e_ref=eps)
    w = o.matsubara(o.FERMION, 16, beta)
    assert np.max(np.abs(F - 1.0 / (1j * w[:, None] - eps[None, :]))) < 1e-13


def adler_wiser(Mq, eps, kmq_q, beta, s, niw):
    """P0_IJ(q, i nu) = s sum_k sum_nm M^I conj(M^J) (f_n - f_m)/(i nu - e_n + e_m),
    the Matsubara transform of eq. irpol with G0 written out by hand
    (degenerate nu = 0 limit: beta f (1 - f))."""
    nu = 2 * np.pi * np.arange(niw) / beta
    NI = Mq[0].shape[0]
    out = np.zeros((niw, NI, NI), dtype=complex)
    for k, Mk in enumerate(Mq):
        kq = kmq_q[k]
        en, em = eps[k, :Mk.shape[1]], eps[kq, :Mk.shape[2]]
        fn, fm = 1 / (np.exp(beta * en) + 1), 1 / (np.exp(beta * em) + 1)
        for a in range(niw):
            de = en[:, None] - em[None, :]
            with np.errstate(divide="ignore", invalid="ignore"):
                ratio = (fn[:, None] - fm[None, :]) / (1j * nu[a] - de)
            if a == 0:
                # nu = 0, e_n = e_m: the ratio tends to -df/de = beta f (1 - f)
                deg = np.abs(de) < 1e-12
                ratio = np.where(deg, beta * fn[:, None] * (1 - fn[:, None]), ratio)
            A = Mk.reshape(NI, -1)
            out[a] += (A * ratio.reshape(-1)) @ A.conj().T
    return s * out


def test_boson_transform_of_P_converges_to_adler_wiser():
    cfg = gi.tiny(grid=(2, 1, 1), nocc=2, nemp=2, ni=3, beta=8.0)
    g = gi.MGenerator(cfg)
    eps = gi.band_energies(cfg)
    kmq = gi.kmq_table(cfg)
    q = 1
    Mq = g.q_blocks(q)
    ref = adler_wiser(Mq, eps, kmq[q], cfg.beta, cfg.scale, 6)
    errs = []
    for n in (16, 32, 64):
        t = np.linspace(0, cfg.beta, n + 1)
        G = o.green0(eps, gi.band_counts(cfg), t, cfg.beta)
        P = o.polarization(Mq, G, kmq[q], cfg.scale)
        Piw = o.tau_to_iw(P, t, cfg.beta, o.BOSON, 6)
        errs.append(np.max(np.abs(Piw - ref)) / np.max(np.abs(ref)))
    assert errs[-1] < 1e-5
    assert errs[0] / errs[1] > 10 and errs[1] / errs[2] > 12


# ---------------------------------------------------------------------------
# polarization
# ---------------------------------------------------------------------------
def test_polarization_hermitian_mirror_negative():
    cfg = gi.C1
    p = gi.make_problem(cfg)
    g = gi.MGenerator(cfg)
    G = o.green0(p.eps, p.nb, p.tau, cfg.beta)
    for q in (0, 3, 7):
        P = o.polarization(g.q_blocks(q), G, p.kmq[q], cfg.scale)
        scale = np.abs(P).max()
        assert np.abs(P - np.conj(np.swapaxes(P, 1, 2))).max() < 1e-14 * scale
        assert np.abs(P - P[::-1]).max() < 1e-13 * scale          # P(tau) = P(beta - tau)
        ev = np.linalg.eigvalsh(P)
        assert ev.max() < 1e-12 * scale                           # negative semidefinite


def test_polarization_unit_g_is_plain_gram():
    """With G = -1 everywhere g = 1 and P = s sum_k A_k A_k^H (a plain matrix product)."""
    cfg = gi.tiny(grid=(2, 2, 1), nocc=2, nemp=1, ni=7)
    g = gi.MGenerator(cfg)
    kmq = gi.kmq_table(cfg)
    G = -np.ones((cfg.nk, 3, cfg.ntau + 1))
    q = 2
    Mq = g.q_blocks(q)
    P = o.polarization(Mq, G, kmq[q], cfg.scale)
    ref = cfg.scale * sum(m.reshape(7, -1) @ m.reshape(7, -1).conj().T for m in Mq)
    assert np.abs(P - ref[None]).max() < 1e-14 * np.abs(ref).max()


def test_polarization_literal_loops():
    cfg = gi.tiny(grid=(2, 1, 1), nocc=2, nemp=1, ni=3, ntau=6)
    p = gi.make_problem(cfg)
    g = gi.MGenerator(cfg, symmetric=False)
    G = o.green0(p.eps, p.nb, p.tau, cfg.beta)
    N = p.tau.size
    for q in range(cfg.nk):
        Mq = g.q_blocks(q)
        P = o.polarization(Mq, G, p.kmq[q], cfg.scale)
        for i in range(N):
            for I in range(3):
                for J in range(3):
                    acc = 0j
                    for k in range(cfg.nk):
                        kq = p.kmq[q, k]
                        for n in range(3):
                            for m in range(3):
                                acc += (Mq[k][I, n, m] * np.conj(Mq[k][J, n, m])
                                        * G[k, n, i] * G[kq, m, N - 1 - i])
                    assert abs(cfg.scale * acc - P[i, I, J]) < 1e-13 * (1 + abs(acc))


# ---------------------------------------------------------------------------
# screen
# ---------------------------------------------------------------------------
def test_screen_single_basis_function_closed_form():
    P = np.array([[[-0.7]], [[-0.2 + 0.0j]]], dtype=complex)
    v = np.array([3.0])
    W, R = o.screen(P, v)
    ref = v[0] ** 2 * P[:, 0, 0] / (1 - v[0] * P[:, 0, 0])
    assert np.abs(W[:, 0, 0] - ref).max() < 1e-14
    assert np.abs(R[:, 0, 0] - (ref - v[0] ** 2 * P[:, 0, 0])).max() < 1e-14


def test_screen_scalar_times_identity():
    v = 4 * np.pi / (0.1 + 0.09 * np.arange(6))
    p = -0.37
    P = (p * np.eye(6))[None].astype(complex)
    W, _ = o.screen(P, v)
    assert np.abs(W[0] - np.diag(v ** 2 * p / (1 - v * p))).max() < 1e-12 * np.abs(W).max()


def test_screen_dyson_residual():
    rng = np.random.default_rng(3)
    n = 9
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    P = -(A @ A.conj().T)[None] / n
    v = rng.uniform(0.5, 3, n)
    W, _ = o.screen(P, v)
    V = np.diag(v)
    resid = W[0] - (V @ P[0] @ V + V @ P[0] @ W[0])
    assert np.abs(resid).max() < 1e-12 * np.abs(W).max()


# ---------------------------------------------------------------------------
# one-pole toy: a3..a7 end to end against closed forms
# ---------------------------------------------------------------------------
def test_one_pole_toy_closed_forms():
    """N_k = 1, bands v (eps_v < 0) and c (eps_c > 0), NI = 1, M_cv = M_vc = a.

    P(i nu) = -2 a^2 (f_v - f_c) D / (nu^2 + D^2), D = eps_c - eps_v.
    W~(i nu) = -v c / (nu^2 + O^2), c = 2 v a^2 (f_v - f_c) D, O^2 = D^2 + c.
    W~(tau) = -v c cosh(O (tau - beta/2)) / (2 O sinh(beta O / 2)).
    Sigma^c_c(tau) = -a^2 G_v(tau) W~(tau), Sigma^c_v(tau) = -a^2 G_c(tau) W~(tau).
    """
    beta, ev, ec, a, v = 6.0, -0.4, 0.5, 0.6, 2.0
    D = ec - ev
    fv, fc = 1 / (np.exp(beta * ev) + 1), 1 / (np.exp(beta * ec) + 1)
    c = 2 * v * a * a * (fv - fc) * D
    Om = math.sqrt(D * D + c)
    M = np.zeros((1, 2, 2), dtype=complex)
    M[0, 1, 0] = M[0, 0, 1] = a                       # band 0 = v, band 1 = c
    eps = np.array([[ev, ec]])
    errs = []
    for nint, niw in ((40, 200), (80, 400)):
        t = np.linspace(0, beta, nint + 1)
        G = o.green0(eps, np.array([2]), t, beta)
        P = o.polarization([M], G, np.array([0]), -1.0)
        Piw = o.tau_to_iw(P, t, beta, o.BOSON, niw)
        nu = o.matsubara(o.BOSON, niw, beta)
        Pex = -2 * a * a * (fv - fc) * D / (nu ** 2 + D ** 2)
        W, R = o.screen(Piw, np.array([v]))
        Wex = -v * c / (nu ** 2 + Om ** 2)
        Wt = o.wt_tau(R, P, np.array([v]), t, beta)
        Wtex = -v * c * np.cosh(Om * (t - beta / 2)) / (2 * Om * np.sinh(beta * Om / 2))
        sig = o.sigma_c([M], G, np.array([0]), Wt, -1.0)
        sigex_c = -a * a * G[0, 0] * Wtex
        sigex_v = -a * a * G[0, 1] * Wtex
        sigiw = o.tau_to_iw(sig[0].T, t, beta, o.FERMION, 8)
        # Sigma_c(tau) = (K0/2) [e^{-O beta/2} e^{(O - ev) tau} + e^{O beta/2} e^{-(O + ev) tau}],
        # K0 = -a^2 (1 - f_v) v c / (2 O sinh(beta O / 2)); each exponential transforms as
        # int_0^beta e^{(i w + lam) tau} dtau = (-e^{lam beta} - 1) / (i w + lam)
        K0 = -a * a * (1 - fv) * v * c / (2 * Om * np.sinh(beta * Om / 2))
        w = o.matsubara(o.FERMION, 8, beta)
        ex_c = 0
        for lam, pre in ((Om - ev, np.exp(-Om * beta / 2)), (-(Om + ev), np.exp(Om * beta / 2))):
            ex_c = ex_c + pre * (-np.exp(lam * beta) - 1) / (1j * w + lam)
        ex_c = 0.5 * K0 * ex_c
        errs.append((np.abs(Piw[:, 0, 0] - Pex).max() / abs(Pex).max(),
                     np.abs(W[:, 0, 0] - Wex).max() / abs(Wex).max(),
                     np.abs(Wt[:, 0, 0] - Wtex).max() / abs(Wtex).max(),
                     max(np.abs(sig[0, 1] - sigex_c).max(), np.abs(sig[0, 0] - sigex_v).max())
                     / np.abs(sigex_c).max(),
                     np.abs(sigiw[:, 1] - ex_c).max() / np.abs(ex_c).max()))
    e1, e2 = np.array(errs[0]), np.array(errs[1])
    assert (e2 < 2e-4).all(), e2
    assert (e1 / e2 > 6).all(), (e1, e2)


def test_sigma_x_two_level_closed_form():
    a, v = 0.8, 1.7
    M = np.zeros((1, 2, 2), dtype=complex)
    M[0, 1, 0] = M[0, 0, 1] = a
    occ = np.array([[0.97, 0.01]])
    sx = o.sigma_x([M], occ, np.array([0]), np.array([v]), -1.0)
    # Sigma^x_c = s f_v a^2 v, Sigma^x_v = s f_c a^2 v
    assert sx[0, 1] == pytest.approx(-occ[0, 0] * a * a * v, rel=1e-15)
    assert sx[0, 0] == pytest.approx(-occ[0, 1] * a * a * v, rel=1e-15)


def test_sigma_c_literal_loops():
    cfg = gi.tiny(grid=(2, 1, 1), nocc=2, nemp=1, ni=3, ntau=6)
    p = gi.make_problem(cfg)
    g = gi.MGenerator(cfg, symmetric=False)
    G = o.green0(p.eps, p.nb, p.tau, cfg.beta)
    rng = np.random.default_rng(5)
    N = p.tau.size
    Wt = rng.normal(size=(N, 3, 3)) + 1j * rng.normal(size=(N, 3, 3))
    Wt = Wt + np.conj(np.swapaxes(Wt, 1, 2))
    q = 1
    Mq = g.q_blocks(q)
    S = o.sigma_c(Mq, G, p.kmq[q], Wt, cfg.scale)
    for k in range(cfg.nk):
        kq = p.kmq[q, k]
        for n in range(3):
            for i in range(N):
                acc = 0j
                for m in range(3):
                    for I in range(3):
                        for J in range(3):
                            acc += G[kq, m, i] * np.conj(Mq[k][I, n, m]) * Wt[i, I, J] * Mq[k][J, n, m]
                assert abs(cfg.scale * acc.real - S[k, n, i]) < 1e-13 * (1 + abs(acc))


# ---------------------------------------------------------------------------
# Dyson and the chemical potential
# ---------------------------------------------------------------------------
def test_dyson_static_self_energy_is_shifted_G0():
    cfg = gi.tiny(grid=(2, 1, 1), nocc=2, nemp=2, beta=15.0, ntau=20, niw=64)
    p = gi.make_problem(cfg)
    shift = np.array([[0.1, -0.05, 0.2, 0.0], [0.03, 0.0, -0.1, 0.05]])
    sig0 = np.zeros(p.eps.shape + (cfg.niw_f,), dtype=complex)
    d = o.dyson(p.eps, p.nb, shift, sig0, cfg.beta, p.tau, p.n_target)
    E = p.eps + shift - d["mu"]
    assert np.abs(d["G_tau"] - o.green0_tau(E, p.tau, cfg.beta)).max() < 1e-14
    assert d["N"] == pytest.approx(p.n_target, abs=1e-10)
    assert (-d["G_tau"][:, :, -1]).sum() == pytest.approx(d["N"], abs=1e-12)


def test_dyson_one_band_mu_closed_form():
    beta, eps, n = 12.0, 0.3, 0.27
    tau = np.linspace(0, beta, 17)
    d = o.dyson(np.array([[eps]]), np.array([1]), np.zeros((1, 1)),
                np.zeros((1, 1, 8), dtype=complex), beta, tau, n)
    assert d["mu"] == pytest.approx(eps - math.log(1 / n - 1) / beta, abs=1e-12)


def test_dyson_sum_rule_and_jump_with_dynamic_sigma():
    cfg = gi.tiny(grid=(2, 1, 1), nocc=2, nemp=2, beta=15.0, ntau=20, niw=64)
    p = gi.make_problem(cfg)
    w = o.matsubara(o.FERMION, cfg.niw_f, cfg.beta)
    # a causal one-pole self-energy 0.2 / (i w - 0.4)
    sig = np.broadcast_to(0.2 / (1j * w - 0.4), p.eps.shape + (cfg.niw_f,)).copy()
    d = o.dyson(p.eps, p.nb, np.zeros_like(p.eps), sig, cfg.beta, p.tau, p.n_target)
    G = d["G_tau"]
    assert np.abs(G[:, :, 0] + G[:, :, -1] + 1.0).max() < 1e-13   # G(0+) + G(beta-) = -1
    assert (-G[:, :, -1]).sum() == pytest.approx(d["N"], abs=1e-10)
    assert d["N"] == pytest.approx(p.n_target, abs=1e-9)
    assert (G < 1e-12).all()                                       # G(tau) <= 0


# ---------------------------------------------------------------------------
# brute force on the real-space toy
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def toy():
    return Toy()


def _toy_G(toy):
    return toy.G_bands(lambda e: o.green0_tau(e, toy.tau, toy.beta))


def test_bruteforce_polarization(toy):
    Gb = _toy_G(toy)
    Pr = toy.P_real(Gb)
    for q in range(NK):
        ref = toy.project_pair(Pr, q)
        got = o.polarization(toy.M[q], Gb, toy.kmq[q], toy.s)
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    # cross-q projections vanish (translation invariance of the toy)
    cross = np.einsum("ir,trs,js->tij", toy.pw[0].conj(), Pr, toy.pw[1])
    assert np.abs(cross).max() < 1e-12 * np.abs(Pr).max()


def test_bruteforce_screen(toy):
    Gb = _toy_G(toy)
    Pr = toy.P_real(Gb)
    niw = 5
    Pr_iw = o.tau_to_iw(Pr, toy.tau, toy.beta, o.BOSON, niw)
    vr = toy.v_real()
    for q in range(NK):
        Plib = o.polarization(toy.M[q], Gb, toy.kmq[q], toy.s)
        Piw = o.tau_to_iw(Plib, toy.tau, toy.beta, o.BOSON, niw)
        W, _ = o.screen(Piw, toy.v_lib[q])
        for a in range(niw):
            Wr = np.linalg.solve(np.eye(8) - vr @ Pr_iw[a], vr @ Pr_iw[a] @ vr)
            ref = toy.project_pair(Wr, q) / 64.0
            assert np.abs(W[a] - ref).max() < 1e-11 * np.abs(ref).max()


def test_bruteforce_sigma_c_and_sigma_x(toy):
    Gb = _toy_G(toy)
    Gr = toy.G_real(Gb)
    rng = np.random.default_rng(11)
    N = toy.tau.size
    Wlib = []
    for q in range(NK):
        A = rng.normal(size=(N, 4, 4)) + 1j * rng.normal(size=(N, 4, 4))
        Wlib.append(A + np.conj(np.swapaxes(A, 1, 2)))
    Wr = toy.W_real_from_lib(Wlib)
    Sr = -Gr * Wr
    got = sum(o.sigma_c(toy.M[q], Gb, toy.kmq[q], Wlib[q], toy.s, full=True) for q in range(NK))
    gotd = sum(o.sigma_c(toy.M[q], Gb, toy.kmq[q], Wlib[q], toy.s) for q in range(NK))
    for k in range(NK):
        ref = np.moveaxis(toy.project_bands(Sr, k), 0, -1)          # [n, n', tau]
        assert np.abs(got[k] - ref).max() < 1e-12 * np.abs(ref).max()
        assert np.abs(gotd[k] - np.real(np.einsum("nnt->nt", ref))).max() < 1e-12 * np.abs(ref).max()
    # exchange: Sigma^x(r, r') = -rho(r, r') v(r, r'), rho = G(0-) = -G(beta-)
    occ = -Gb[:, :, -1]
    rho = np.einsum("knr,kn,kns->rs", toy.psi, occ, toy.psi.conj())
    Sx = -rho * toy.v_real()
    gx = sum(o.sigma_x(toy.M[q], occ, toy.kmq[q], toy.v_lib[q], toy.s, full=True) for q in range(NK))
    for k in range(NK):
        ref = toy.project_bands(Sx, k)
        assert np.abs(gx[k] - ref).max() < 1e-12 * np.abs(ref).max()


# ---------------------------------------------------------------------------
# planted mistakes: each plausible slip in the oracle's P or Sigma fails a pin
# ---------------------------------------------------------------------------
def _mutant_polarization(kind):
    def P(Mq, G, kmq_q, s):
        ntau = G.shape[2]
        NI = Mq[0].shape[0]
        out = np.zeros((ntau, NI, NI), dtype=complex)
        for k, Mk in enumerate(Mq):
            nn, nm = Mk.shape[1:]
            kq = kmq_q[k]
            A = Mk.reshape(NI, -1)
            for i in range(ntau):
                j = i if kind == "same_tau" else ntau - 1 - i
                g = np.outer(G[k, :nn, i], G[kq, :nm, j]).reshape(-1)
                if kind == "conj_left":
                    out[i] += (A.conj() * g) @ A.T
                else:
                    out[i] += (A * g) @ A.conj().T
        fac = {"no_nk": s * len(Mq), "sign": -s}.get(kind, s)
        return fac * out
    return P


@pytest.mark.parametrize("kind", ["same_tau", "conj_left", "no_nk", "sign"])
def test_planted_polarization_mistakes_are_caught(toy, kind):
    Gb = _toy_G(toy)
    Pr = toy.P_real(Gb)
    bad = _mutant_polarization(kind)
    worst = 0.0
    for q in range(NK):
        ref = toy.project_pair(Pr, q)
        got = bad(toy.M[q], Gb, toy.kmq[q], toy.s)
        worst = max(worst, np.abs(got - ref).max() / np.abs(ref).max())
    assert worst > 1e-3


# ---------------------------------------------------------------------------
# analytic continuation (Pade) and quasiparticle energies
# ---------------------------------------------------------------------------
_POLES = np.array([-0.7, 0.2, 1.1])
_RES = np.array([0.05, 0.1, 0.03])


def _rational(z):
    """A causal three-pole self-energy sum_i r_i / (z - p_i) (r_i > 0)."""
    return np.sum(_RES / (np.asarray(z)[..., None] - _POLES), axis=-1)


@pytest.mark.parametrize("n_pade", [6, 7, 10, 24])
def test_pade_reproduces_a_rational_self_energy(n_pade):
    """Three poles make a [2/3] rational function: six Matsubara points determine it, and the
    continued fraction through them (or more) reproduces it on the real axis."""
    beta = 50.0
    z = o.matsubara_points(n_pade, beta)
    a = o.pade_coefficients(z, _rational(z)[None])
    w = np.linspace(-2.0, 2.0, 81) + 0.01j
    c = o.pade_eval(z, a, w[None])[0]
    assert np.max(np.abs(c - _rational(w)) / np.abs(_rational(w))) < 1e-8
    # interpolation property at the data points themselves
    assert np.allclose(o.pade_eval(z, a, z[None])[0], _rational(z), rtol=1e-12, atol=0)


def test_pade_derivative_matches_closed_form():
    beta, n = 50.0, 10
    z = o.matsubara_points(n, beta)
    a = o.pade_coefficients(z, _rational(z)[None])
    w = np.linspace(-1.5, 1.5, 7) + 0.05j
    c, dc = o.pade_eval_and_derivative(z, a, w[None])
    exact = -np.sum(_RES / (w[:, None] - _POLES) ** 2, axis=-1)
    assert np.allclose(dc[0], exact, rtol=1e-7, atol=0)


def test_qp_energy_one_pole_closed_form():
    """Sigma(z) = r / (z - p): x = e0 + r / (x - p) is a quadratic; Newton from e0 reaches the root
    nearest e0."""
    beta, p, r = 50.0, 0.8, 0.04
    e0 = np.array([[-0.5, 0.3, 1.5, 0.9]])
    w = (2 * np.arange(32) + 1) * np.pi / beta
    sig = np.broadcast_to(r / (1j * w - p), (1, 4, 32))
    E, ok = o.qp_energies(e0, [4], np.zeros_like(e0), sig, 0.0, beta, 8, 0.0)
    assert ok.all()
    for x, e in zip(E[0], e0[0]):
        roots = np.roots([1.0, -(e + p), e * p - r])
        assert abs(x - roots[np.argmin(np.abs(roots - e))]) < 1e-12
    # mu shifts the energies rigidly
    E2, _ = o.qp_energies(e0 + 0.25, [4], np.zeros_like(e0), sig, 0.25, beta, 8, 0.0)
    assert np.allclose(E2, E + 0.25, rtol=0, atol=1e-12)


def test_spectral_function_sum_rule_and_peak():
    """A(w) of a causal self-energy integrates to one; a static self-energy gives a Lorentzian of
    half-width eta at e0 + Sigma."""
    beta, eta = 50.0, 0.02
    w = (2 * np.arange(32) + 1) * np.pi / beta
    sig = (0.04 / (1j * w - 0.8))[None, None, :]
    om = np.linspace(-40.0, 40.0, 400001)
    A = o.spectral(np.array([[0.3]]), np.zeros((1, 1)), sig, 0.0, beta, 8, eta, om)[0, 0]
    assert abs(np.trapezoid(A, om) - 1.0) < 2e-3
    static = np.full((1, 1, 8), 0.1 + 0j)
    A0 = o.spectral(np.array([[0.3]]), np.zeros((1, 1)), static, 0.0, beta, 1, eta, om)[0, 0]
    lor = eta / np.pi / ((om - 0.4) ** 2 + eta ** 2)
    assert np.max(np.abs(A0 - lor)) < 1e-12 * lor.max()


def test_qp_gap_orders_states():
    E = np.array([[0.3, -0.2, 9.0], [0.1, -0.5, 0.7]])
    assert o.qp_gap(E, [2, 3], 2) == pytest.approx(0.1 - (-0.2))
    assert o.qp_gap(E, [2, 3], 3) == pytest.approx(0.3 - 0.1)


@pytest.mark.parametrize("kind", ["sign", "index", "conj"])
def test_planted_pade_mistakes_are_caught(kind):
    """The rational pin rejects plausible slips in the continued-fraction recursion."""
    beta, n = 50.0, 10
    z = o.matsubara_points(n, beta)
    u = _rational(z)
    g = u.astype(np.complex128).copy()
    a = np.empty_like(g)
    a[0] = g[0]
    for p in range(1, n):
        prev = g[p - 1]
        dz = z[p:] - z[p - 1]
        if kind == "sign":
            dz = -dz
        if kind == "conj":
            prev = np.conj(prev)
        nxt = (prev - g[p:]) / (dz * g[p:])
        if kind == "index":
            nxt = (prev - g[p:]) / (dz * g[p - 1])
        g[p:] = nxt
        a[p] = g[p]
    w = np.linspace(-2.0, 2.0, 81) + 0.01j
    c = o.pade_eval(z, a[None], w[None])[0]
    assert np.max(np.abs(c - _rational(w)) / np.abs(_rational(w))) > 1e-3


# ---------------------------------------------------------------------------
# continuous-pole expansion
# ---------------------------------------------------------------------------
def test_cpe_basis_matches_quadrature():
    """The closed form of Phi_l(z) = int h_l(w) / (w - z) dw against numerical quadrature."""
    wg = o.cpe_grid(-3.0, 3.0, 41)
    z = np.array([0.3 + 0.2j, -1.0 + 0.05j, 2.0 + 1.0j, 0.0 + 0.8j])
    phi, dphi = o.cpe_phi(wg, z, derivative=True)
    for l in (0, 17, 38):
        def h(w):
            return np.interp(w, wg[l:l + 3], [0.0, 1.0, 0.0])
        for i, zz in enumerate(z):
            den = lambda w: (w - zz.real) ** 2 + zz.imag ** 2  # noqa: E731
            re = quad(lambda w: h(w) * (w - zz.real) / den(w), wg[l], wg[l + 2], points=[wg[l + 1]])[0]
            im = quad(lambda w: h(w) * zz.imag / den(w), wg[l], wg[l + 2], points=[wg[l + 1]])[0]
            assert abs(phi[i, l] - (re + 1j * im)) < 1e-10
            # derivative: int h / (w - z)^2
            d2 = lambda w: (w - zz) ** 2  # noqa: E731
            dre = quad(lambda w: (h(w) / d2(w)).real, wg[l], wg[l + 2], points=[wg[l + 1]])[0]
            dim = quad(lambda w: (h(w) / d2(w)).imag, wg[l], wg[l + 2], points=[wg[l + 1]])[0]
            assert abs(dphi[i, l] - (dre + 1j * dim)) < 1e-8


def test_cpe_recovers_an_exact_expansion():
    """Data generated by non-negative coefficients are fitted back; the continued self-energy is the
    spectral integral of the piecewise-linear Im Sigma."""
    beta = 50.0
    wg = o.cpe_grid(-3.0, 3.0, 41)
    a_true = np.zeros(39)
    a_true[[10, 11, 12, 25, 26]] = [0.02, 0.05, 0.02, 0.03, 0.01]
    B = o.cpe_basis(wg, beta, 64)
    y = B @ a_true
    a = o.cpe_fit(wg, beta, (y[:64] + 1j * y[64:])[None], 1e-14)[0]
    assert np.all(a >= 0)
    assert np.linalg.norm(a - a_true) < 1e-6 * np.linalg.norm(a_true)
    z = 0.4 + 0.05j
    im_sig = lambda w: -np.interp(w, wg[1:-1], a_true, left=0.0, right=0.0)  # noqa: E731
    d = lambda w: (w - z.real) ** 2 + z.imag ** 2  # noqa: E731
    re = quad(lambda w: im_sig(w) * (w - z.real) / d(w), -3, 3, points=list(wg[9:14]) + list(wg[24:28]),
              limit=200)[0] / np.pi
    im = quad(lambda w: im_sig(w) * z.imag / d(w), -3, 3, points=list(wg[9:14]) + list(wg[24:28]),
              limit=200)[0] / np.pi
    assert abs(o.cpe_sigma(wg, a, np.array(z)) - (re + 1j * im)) < 1e-8


def test_cpe_one_pole_weight_causality_and_qp():
    """Sigma = r / (z - p): the fit is causal (a >= 0, Im Sigma(w) <= 0), carries the pole's weight r,
    satisfies the optimality conditions of the constrained problem, and gives the quasiparticle
    energy of the exact self-energy to the resolution of the grid."""
    beta, r, p, ridge = 50.0, 0.04, 0.8, 1e-10
    wg = o.cpe_grid(-3.0, 3.0, 61)
    w = (2 * np.arange(64) + 1) * np.pi / beta
    sig = (r / (1j * w - p))[None, None, :]
    a = o.cpe_fit(wg, beta, sig, ridge)[0, 0]
    assert np.all(a >= 0)
    dw = wg[1] - wg[0]
    assert abs(np.sum(a) * dw / np.pi - r) < 0.03 * r
    B = o.cpe_basis(wg, beta, 64)
    lam = ridge * np.max(np.sum(B * B, axis=0))
    g = B.T @ (B @ a - np.concatenate([sig[0, 0].real, sig[0, 0].imag])) + lam * a
    scale = np.linalg.norm(B.T @ np.concatenate([sig[0, 0].real, sig[0, 0].imag]))
    assert np.all(g[a > 0] < 1e-6 * scale) and np.all(g[a > 0] > -1e-6 * scale)
    assert np.all(g[a == 0] > -1e-6 * scale)
    e0 = np.array([[0.3]])
    E, ok, _ = o.qp_energies_cpe(e0, [1], np.zeros_like(e0), sig, 0.0, beta, wg, ridge, 0.02)
    roots = np.roots([1.0, -(0.3 + p), 0.3 * p - r])
    exact = roots[np.argmin(np.abs(roots - 0.3))]
    assert ok.all() and abs(E[0, 0] - exact) < 2e-3


# ---------------------------------------------------------------------------
# inverse bosonic transform of W~: the negative-frequency term
# ---------------------------------------------------------------------------
# For a Hermitian P(tau), P(-i nu) = P(i nu)^H, and with a real diagonal v the same holds for
# W~ and R = W~ - v P v.  The truncated inverse sum must therefore pair each R(i nu_n) with
# R(i nu_n)^H at -nu_n.  Two facts fix that pairing independently of the oracle's formula:
# the result is Hermitian at every tau for any Hermitian P(tau) (also without the tau mirror),
# and the forward transform of the result at +nu_m and at -nu_m returns R(i nu_m) and
# R(i nu_m)^H.
def _mutant_boson_inverse(kind):
    """A literal loop of the inverse bosonic sum whose partner of R_n is R_n^H ("RH", the
    reading) or a planted slip (R^T, conj R, R)."""
    def inv(R, tau, beta, add_tau=None):
        niw = R.shape[0]
        nu = o.matsubara(o.BOSON, niw, beta)
        partner = {"RH": np.conj(np.swapaxes(R, 1, 2)), "RT": np.swapaxes(R, 1, 2),
                   "conjR": np.conj(R), "R": R}[kind]
        out = np.zeros((tau.size,) + R.shape[1:], dtype=complex)
        for i, t in enumerate(tau):
            out[i] = R[0]
            for n in range(1, niw):
                out[i] += np.exp(-1j * nu[n] * t) * R[n] + np.exp(1j * nu[n] * t) * partner[n]
        out /= beta
        return out if add_tau is None else out + add_tau
    return inv


def _screen_chain_without_mirror():
    """W~(tau) of one q for a Hermitian P(tau) without P(tau) = P(beta - tau) (independent M)."""
    cfg = gi.tiny(grid=(3, 1, 1), nocc=2, nemp=3, ni=6, ntau=24, beta=8.0, niw=10)
    p = gi.make_problem(cfg)
    g = gi.MGenerator(cfg, symmetric=False)
    G = o.green0(p.eps, p.nb, p.tau, cfg.beta)
    q = 1
    P = o.polarization(g.q_blocks(q), G, p.kmq[q], cfg.scale)
    Piw = o.tau_to_iw(P, p.tau, cfg.beta, o.BOSON, cfg.niw_b)
    _, R = o.screen(Piw, p.v[q])
    return cfg, p, q, P, R


def test_wt_tau_hermitian_without_tau_mirror():
    cfg, p, q, P, R = _screen_chain_without_mirror()
    # the inputs are generic: P(tau) Hermitian but not mirror symmetric, R neither Hermitian,
    # real nor symmetric, so no partner other than R^H gives a Hermitian sum
    assert np.abs(P - np.conj(np.swapaxes(P, 1, 2))).max() < 1e-13 * np.abs(P).max()
    assert np.abs(P - P[::-1]).max() > 1e-3 * np.abs(P).max()
    for other in (np.conj(np.swapaxes(R, 1, 2)), np.conj(R), np.swapaxes(R, 1, 2)):
        assert np.abs(R[1:] - other[1:]).max() > 1e-3 * np.abs(R[1:]).max()
    Wt = o.wt_tau(R, P, p.v[q], p.tau, cfg.beta)
    herm = np.abs(Wt - np.conj(np.swapaxes(Wt, 1, 2))).max(axis=(1, 2))
    assert herm.max() < 1e-12 * np.abs(Wt).max()


def test_boson_inverse_round_trip_both_frequency_signs():
    rng = np.random.default_rng(5)
    beta, niw, n = 10.0, 6, 4
    R = rng.normal(size=(niw, n, n)) + 1j * rng.normal(size=(niw, n, n))
    tau = np.linspace(0.0, beta, 2001)
    f = o.iw_to_tau_boson_herm(R, tau, beta)
    pos = o.tau_to_iw(f, tau, beta, o.BOSON, niw)                   # int e^{+i nu tau} f
    neg = np.conj(o.tau_to_iw(np.conj(f), tau, beta, o.BOSON, niw))  # int e^{-i nu tau} f
    scale = np.abs(R).max()
    assert np.abs(pos - R).max() < 1e-6 * scale
    assert np.abs(neg[1:] - np.conj(np.swapaxes(R[1:], 1, 2))).max() < 1e-6 * scale
    # the constant term appears once: at nu = 0 both signs give R_0
    assert np.abs(neg[0] - R[0]).max() < 1e-6 * scale


@pytest.mark.parametrize("kind", ["RT", "conjR", "R"])
def test_planted_boson_inverse_mistakes_are_caught(kind):
    bad = _mutant_boson_inverse(kind)
    # the planted copy agrees with the oracle when its partner is the right one
    cfg, p, q, P, R = _screen_chain_without_mirror()
    good = _mutant_boson_inverse("RH")(R, p.tau, cfg.beta)
    assert np.abs(good - o.iw_to_tau_boson_herm(R, p.tau, cfg.beta)).max() < 1e-12 * np.abs(good).max()
    # Hermiticity pin
    v = np.asarray(p.v[q])
    Wt = bad(R, p.tau, cfg.beta, add_tau=v[None, :, None] * P * v[None, None, :])
    herm = np.abs(Wt - np.conj(np.swapaxes(Wt, 1, 2))).max()
    assert herm > 1e-4 * np.abs(Wt).max()
    # round-trip pin
    rng = np.random.default_rng(5)
    beta, niw, n = 10.0, 6, 4
    Rr = rng.normal(size=(niw, n, n)) + 1j * rng.normal(size=(niw, n, n))
    tau = np.linspace(0.0, beta, 401)
    f = bad(Rr, tau, beta)
    neg = np.conj(o.tau_to_iw(np.conj(f), tau, beta, o.BOSON, niw))
    assert np.abs(neg[1:] - np.conj(np.swapaxes(Rr[1:], 1, 2))).max() > 1e-2 * np.abs(Rr).max()


# ---------------------------------------------------------------------------
# gap proxy on a hand-built level list
# ---------------------------------------------------------------------------
def test_gap_proxy_hand_built_levels():
    # two k points, three bands, the third band of k = 1 absent (Nb_1 = 2, its entries are
    # ignored).  E^QP = eps + Sigma_static + Re Sigma^c(i w_0) - mu:
    eps = np.array([[-0.50, 0.10, 0.90], [-0.30, 0.45, 99.0]])
    stat = np.array([[0.05, -0.02, 0.00], [0.00, 0.01, -99.0]])
    sc0 = np.array([[0.01 + 5j, 0.00 - 1j, 0.03 + 0j], [-0.02 + 0j, 0.00 + 2j, 0.0 + 0j]])
    mu = 0.2
    nb = np.array([3, 2])
    # levels before the common -mu: k0: -0.44, 0.08, 0.93; k1: -0.32, 0.46
    # ascending: -0.44, -0.32, 0.08, 0.46, 0.93 (the imaginary parts play no role)
    want = {1: -0.32 - (-0.44), 2: 0.08 - (-0.32), 3: 0.46 - 0.08, 4: 0.93 - 0.46}
    for n_target, N in ((1.0, 1), (2.4, 2), (2.6, 3), (4.0, 4)):
        got = o.gap_proxy(eps, nb, stat, sc0, mu, n_target)
        assert got == pytest.approx(want[N], abs=1e-14)


def test_planted_gap_proxy_index_slip_is_caught():
    eps = np.array([[-0.50, 0.10, 0.90], [-0.30, 0.45, 99.0]])
    stat = np.zeros_like(eps)
    sc0 = np.zeros(eps.shape, dtype=complex)
    nb = np.array([3, 2])

    def slipped(eps, nb, sig_static, sigc_iw0, mu, n_target):
        mask = np.arange(eps.shape[1])[None, :] < np.asarray(nb)[:, None]
        e = np.sort((eps + sig_static + np.real(sigc_iw0) - mu)[mask])
        N = int(round(n_target))
        return float(e[N + 1] - e[N])

    ref = o.gap_proxy(eps, nb, stat, sc0, 0.0, 2.0)
    assert ref == pytest.approx(0.10 - (-0.30), abs=1e-14)
    assert abs(slipped(eps, nb, stat, sc0, 0.0, 2.0) - ref) > 0.01


# ---------------------------------------------------------------------------
# Dyson equation with off-diagonal band matrices
# ---------------------------------------------------------------------------
def _hermitian(rng, n, scale):
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    return 0.5 * scale * (A + A.conj().T)


def test_dyson_matrix_reduces_to_the_diagonal_dyson():
    cfg = gi.tiny(grid=(2, 1, 1), nocc=2, nemp=2, beta=15.0, ntau=20, niw=64)
    p = gi.make_problem(cfg)
    rng = np.random.default_rng(4)
    w = o.matsubara(o.FERMION, cfg.niw_f, cfg.beta)
    stat = rng.uniform(-0.1, 0.1, size=p.eps.shape)
    sig = 0.2 / (1j * w[None, None, :] - rng.uniform(-0.5, 0.5, size=p.eps.shape + (1,)))
    d = o.dyson(p.eps, p.nb, stat, sig, cfg.beta, p.tau, p.n_target)
    nk, nb = p.eps.shape
    S0 = np.zeros((nk, nb, nb), dtype=complex)
    S = np.zeros((nk, nb, nb, cfg.niw_f), dtype=complex)
    for k in range(nk):
        S0[k] = np.diag(stat[k])
        for n in range(nb):
            S[k, n, n] = sig[k, n]
    m = o.dyson_matrix(p.eps, p.nb, S0, S, cfg.beta, p.tau, p.n_target)
    assert m["mu"] == pytest.approx(d["mu"], abs=1e-12)
    assert abs(m["N"] - d["N"]) < 1e-10
    diag = np.einsum("knnt->knt", m["G_tau"])
    assert np.abs(diag - d["G_tau"]).max() < 1e-12
    off = m["G_tau"] - np.einsum("knt,nm->knmt", diag, np.eye(nb))
    assert np.abs(off).max() < 1e-14


def _static_case(niw, seed=8):
    beta, nb = 12.0, 4
    rng = np.random.default_rng(seed)
    eps = np.array([[-0.6, -0.2, 0.3, 0.8]])
    S0 = _hermitian(rng, nb, 0.15)[None]                       # complex off-diagonal coupling
    tau = np.linspace(0.0, beta, 25)
    return beta, nb, eps, S0, tau, np.zeros((1, nb, nb, niw), dtype=complex)


def test_dyson_matrix_static_closed_form():
    """Static Hermitian Sigma: G(k, i w) = V diag(1 / (i w + mu - lambda)) V^H and
    G(tau) = V diag(G0(lambda - mu, tau)) V^H with H0 = V diag(lambda) V^H (textbook), the tau
    side within the O(1/niw) truncation of the Matsubara sum (error falls ~4x for 4x niw), and
    mu placing sum_j n_F(lambda_j - mu) at the target within that truncation."""
    errs = []
    for niw in (256, 1024):
        beta, nb, eps, S0, tau, S = _static_case(niw)
        H0 = np.diag(eps[0]) + S0[0]
        lam, V = np.linalg.eigh(H0)
        n_target = 2.3
        m = o.dyson_matrix(eps, np.array([nb]), S0, S, beta, tau, n_target)
        mu = m["mu"]
        w = o.matsubara(o.FERMION, niw, beta)
        Gex = np.einsum("ij,jn,kj->ikn", V, 1.0 / (1j * w[None, :] + mu - lam[:, None]), V.conj())
        assert np.abs(m["G_iw"][0] - Gex).max() < 1e-13
        Gt = np.einsum("ij,jt,kj->ikt", V, o.green0_tau(lam - mu, tau, beta), V.conj())
        errs.append((np.abs(m["G_tau"][0] - Gt).max(), abs(o.fermi(lam - mu, beta).sum() - n_target)))
    (e1, n1), (e2, n2) = errs
    assert e2 < 2e-4 and 3.0 < e1 / e2 < 5.0, errs
    assert n2 < 1e-3 and n1 / n2 > 3.0, errs


def test_dyson_matrix_jump_sum_rule_and_hermiticity():
    beta, nb, eps, S0, tau, _ = _static_case(128)
    niw = 128
    w = o.matsubara(o.FERMION, niw, beta)
    rng = np.random.default_rng(2)
    # a causal matrix self-energy B / (i w - p) with B Hermitian positive: Sigma(-i w) = Sigma(i w)^H
    Bm = _hermitian(rng, nb, 0.1)
    Bm = Bm @ Bm.conj().T
    S = (Bm[:, :, None] / (1j * w[None, None, :] - 0.35))[None]
    m = o.dyson_matrix(eps, np.array([nb]), S0, S, beta, tau, 2.0)
    G = m["G_tau"][0]
    assert np.abs(G[:, :, 0] + G[:, :, -1] + np.eye(nb)).max() < 1e-13     # G(0+) + G(beta-) = -1
    assert abs(-np.trace(G[:, :, -1]).real - m["N"]) < 1e-10               # N = -Tr G(beta-)
    assert m["N"] == pytest.approx(2.0, abs=1e-9)
    assert np.abs(G - np.conj(np.swapaxes(G, 0, 1))).max() < 1e-13       # Hermitian at every tau


def test_planted_dyson_matrix_transpose_is_caught():
    """D^T instead of D^H at the negative frequencies (a plausible slip) breaks the static closed form."""
    beta, nb, eps, S0, tau, S = _static_case(256)
    m = o.dyson_matrix(eps, np.array([nb]), S0, S, beta, tau, 2.3)
    H0 = np.diag(eps[0]) + S0[0]
    lam, V = np.linalg.eigh(H0)
    Gt = np.einsum("ij,jt,kj->ikt", V, o.green0_tau(lam - m["mu"], tau, beta), V.conj())
    D = m["G_iw"][0].copy()
    E = np.real(np.diag(H0)) - m["mu"]
    w = o.matsubara(o.FERMION, 256, beta)
    D[np.arange(nb), np.arange(nb), :] -= 1.0 / (1j * w[None, :] - E[:, None])
    ph = np.exp(-1j * np.outer(tau, w))
    bad = (np.tensordot(D, ph.T, axes=([-1], [0]))
           + np.tensordot(np.swapaxes(D, 0, 1), np.conj(ph).T, axes=([-1], [0]))) / beta
    bad[np.arange(nb), np.arange(nb), :] += o.green0_tau(E, tau, beta)
    good_err, bad_err = np.abs(m["G_tau"][0] - Gt).max(), np.abs(bad - Gt).max()
    assert good_err < 1e-3 and bad_err > 10 * good_err, (good_err, bad_err)
