"""Pins of the oracle's tau-domain solvers: the W~ linear system (eq. tildeW, trapezoid increments)
and the G Dyson system on the dense uniform grid (eqs. dysongf, zxjk, zcjk, dysong).

Closed forms fix both: a bosonic one-pole polarization screened in each eigen-channel of v^1/2 B v^1/2,
and a fermionic one-pole self-energy, whose Dyson solution is a two-pole Green's function.  Both
solvers are second-order in the grid spacing (trapezoid rule with the jumps at nodes taken as the
mean of their limits), which the error ratios under halving check; the Matsubara-axis routes of the
oracle converge to the same closed forms, so the two routes agree to discretisation error.
"""
import math

import numpy as np
import pytest

import gwinputs as gi
import oracle as o


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------
def boson_pole(D, t, beta):
    """(1/beta) sum_n -2D/(nu_n^2 + D^2) e^{-i nu_n t} = -cosh(D (t - beta/2)) / sinh(beta D / 2)."""
    return -np.cosh(D * (t - beta / 2)) / np.sinh(beta * D / 2)


def screened_channels(B, v, D, t, beta):
    """W~(t) for P(t) = B boson_pole(D, t) and diagonal v: in each eigen-channel s of S = v^1/2 B v^1/2
    the screened pole is -s (D / W) cosh(W (t - beta/2)) / sinh(beta W / 2), W^2 = D^2 + 2 s D."""
    sv = np.sqrt(v)
    s, U = np.linalg.eigh(sv[:, None] * B * sv[None, :])
    Om = np.sqrt(D * D + 2.0 * s * D)
    w = -s[None, :] * (D / Om[None, :]) * np.cosh(Om[None, :] * (t[:, None] - beta / 2)) \
        / np.sinh(beta * Om[None, :] / 2)
    X = np.einsum("ia,ta,ja->tij", U, w, U.conj())
    return sv[None, :, None] * X * sv[None, None, :]


def two_pole_green(E, c, Om, t, beta):
    """G for G0 at E and Sigma^c(i w) = c / (i w - Om): poles z = roots of (z - E)(z - Om) = c with
    weights (z_a - Om) / (z_a - z_b)."""
    disc = math.sqrt((E - Om) ** 2 + 4.0 * c)
    z = np.array([(E + Om + disc) / 2, (E + Om - disc) / 2])
    w = np.array([(z[0] - Om) / (z[0] - z[1]), (z[1] - Om) / (z[1] - z[0])])
    return sum(w[a] * o.green0_tau(z[a], t, beta) for a in range(2))


def _hermitian_psd(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    return X @ X.conj().T / n


# ---------------------------------------------------------------------------
# W~ tau system
# ---------------------------------------------------------------------------
def test_wt_tau_system_one_pole_second_order():
    """The one-pole toy (two bands, NI = 1): W~(t) = -v c cosh(W (t - beta/2)) / (2 W sinh(beta W / 2))."""
    beta, ev, ec, a, v = 6.0, -0.4, 0.5, 0.6, 2.0
    D = ec - ev
    fv, fc = o.fermi(ev, beta), o.fermi(ec, beta)
    c = 2 * v * a * a * (fv - fc) * D
    Om = math.sqrt(D * D + c)
    M = np.zeros((1, 2, 2), complex)
    M[0, 1, 0] = M[0, 0, 1] = a
    eps = np.array([[ev, ec]])
    errs = []
    for n in (20, 40, 80):
        t = np.linspace(0, beta, n + 1)
        P = o.polarization([M], o.green0(eps, np.array([2]), t, beta), np.array([0]), -1.0)
        W = o.wt_tau_system(P, np.array([v]), t, beta)
        ex = -v * c * np.cosh(Om * (t - beta / 2)) / (2 * Om * np.sinh(beta * Om / 2))
        errs.append(np.abs(W[:, 0, 0] - ex).max() / np.abs(ex).max())
    assert errs[-1] < 2e-3
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.6 < e0 / e1 < 4.4, errs


def test_wt_tau_system_matrix_channels_and_hermiticity():
    """NI = 4 with a non-uniform v: each eigen-channel of v^1/2 B v^1/2 screens its own pole; W~ is
    Hermitian and mirror-symmetric at every tau."""
    beta, D = 5.0, 0.9
    v = np.array([2.0, 1.3, 0.7, 0.4])
    B = _hermitian_psd(4, 11) * 0.3
    errs = []
    for n in (32, 64):
        t = np.linspace(0, beta, n + 1)
        P = B[None] * boson_pole(D, t, beta)[:, None, None]
        W = o.wt_tau_system(P, v, t, beta)
        ex = screened_channels(B, v, D, t, beta)
        errs.append(np.abs(W - ex).max() / np.abs(ex).max())
        assert np.abs(W - np.conj(np.swapaxes(W, 1, 2))).max() < 1e-12 * np.abs(W).max()
        assert np.abs(W - W[::-1]).max() < 1e-10 * np.abs(W).max()
    assert errs[-1] < 2e-3
    assert 3.6 < errs[0] / errs[1] < 4.4, errs


def _mutant_wt_tau_system(P_tau, v, tau, beta, kind):
    """wt_tau_system with one planted mistake: 'Pv' (A = P v), 'flat' (no half increments at the
    ends), 'nowrap' (A(x) at x < 0 read as 0)."""
    tau = np.asarray(tau, dtype=np.float64)
    N, NI = tau.size, v.size
    dt = o.trapezoid_increments(tau)
    if kind == "flat":
        dt = np.full(N, beta / (N - 1))
    x = tau[:, None] - tau[None, :]
    neg = x < 0.0
    x = np.where(neg, x + beta, x)
    Px = o.spline_eval(tau, P_tau, x.reshape(-1)).reshape(N, N, NI, NI)
    if kind == "nowrap":
        Px = np.where(neg[:, :, None, None], 0.0, Px)
    A = Px * v[None, None, None, :] if kind == "Pv" else v[None, None, :, None] * Px
    K = np.moveaxis(-A * dt[None, :, None, None], 1, 2).reshape(N * NI, N * NI) + np.eye(N * NI)
    rhs = v[None, :, None] * P_tau * v[None, None, :]
    return np.linalg.solve(K, rhs.reshape(N * NI, NI)).reshape(N, NI, NI)


@pytest.mark.parametrize("kind", ["Pv", "flat", "nowrap"])
def test_planted_wt_tau_system_mistakes_are_caught(kind):
    beta, D = 5.0, 0.9
    v = np.array([2.0, 1.3, 0.7, 0.4])
    B = _hermitian_psd(4, 11) * 0.3
    errs = []
    for n in (24, 48):
        t = np.linspace(0, beta, n + 1)
        P = B[None] * boson_pole(D, t, beta)[:, None, None]
        ex = screened_channels(B, v, D, t, beta)
        good = o.wt_tau_system(P, v, t, beta)
        bad = _mutant_wt_tau_system(P, v, t, beta, kind)
        assert np.abs(good - ex).max() < 2e-2 * np.abs(ex).max()
        errs.append(np.abs(bad - ex).max() / np.abs(ex).max())
    # a mutant is either wrong outright or loses the second-order convergence
    assert errs[-1] > 1e-2 or errs[0] / errs[1] < 3.0, errs


def test_wt_tau_system_agrees_with_frequency_route():
    """The paper's tau system and the nu-axis screen (with the truncated inverse transform) approach
    the same W~ on a UPM mesh as the points per sub-interval double (m = 3, 6, 12): the tau system at
    second order in the spacing (trapezoid), the nu route at fourth (spline-Filon transform), so their
    difference shrinks with the tau system's error."""
    beta, D = 20.0, 0.7
    v = np.array([1.5, 0.8, 0.5])
    B = _hermitian_psd(3, 5) * 0.2
    et, en, diffs = [], [], []
    for m in (3, 6, 12):
        t = gi.upm_mesh(beta, 2 * m * 3, m)
        P = B[None] * boson_pole(D, t, beta)[:, None, None]
        Wt = o.wt_tau_system(P, v, t, beta)
        Piw = o.tau_to_iw(P, t, beta, o.BOSON, 256)
        _, R = o.screen(Piw, v)
        Wn = o.wt_tau(R, P, v, t, beta)
        ex = screened_channels(B, v, D, t, beta)
        scale = np.abs(ex).max()
        et.append(np.abs(Wt - ex).max() / scale)
        en.append(np.abs(Wn - ex).max() / scale)
        diffs.append(np.abs(Wt - Wn).max() / scale)
    for a, b in zip(et, et[1:]):
        assert 3.0 < a / b < 4.5, et
    for a, b in zip(en, en[1:]):
        assert a / b > 12.0, en
    assert diffs[-1] < 1e-2 and diffs[0] / diffs[-1] > 10.0, diffs


# ---------------------------------------------------------------------------
# G Dyson on the dense uniform grid
# ---------------------------------------------------------------------------
def test_dense_grid_of_upm_mesh():
    t = gi.upm_mesh(40.0, 30, 5)
    td = o.dense_grid(t, 40.0)
    assert td[1] - td[0] == pytest.approx(t[1] - t[0], rel=1e-14)
    assert td[-1] == pytest.approx(40.0, rel=1e-14)
    # every mesh point is a dense point
    idx = np.rint(t / (td[1] - td[0])).astype(int)
    assert np.abs(td[idx] - t).max() < 1e-12 * 40.0


def test_dyson_tau_static_closed_form_second_order():
    """Sigma^c = 0: G is the reference Green's function at the shifted energy E + dsig."""
    beta, E, d = 8.0, 0.3, -0.5
    errs = []
    for n in (32, 64, 128):
        t = np.linspace(0, beta, n + 1)
        td, G, Gm = o.dyson_tau(E, d, np.zeros(n + 1), t, beta)
        errs.append(np.abs(G - o.green0_tau(E + d, td, beta)).max())
        assert np.abs(Gm - G).max() == 0.0
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.6 < e0 / e1 < 4.4, errs


def test_dyson_tau_one_pole_self_energy_second_order():
    """Sigma^c(t) = c G0(Om, t), i.e. c / (i w - Om) on the axis, with a static shift: the two-pole
    Green's function of the poles of 1 / (i w - E - d - c / (i w - Om))."""
    beta, E, d, c, Om = 10.0, 0.4, -0.15, 0.08, -0.6
    errs = []
    for n in (40, 80, 160):
        t = np.linspace(0, beta, n + 1)
        td, G, _ = o.dyson_tau(E, d, c * o.green0_tau(Om, t, beta), t, beta)
        errs.append(np.abs(G - two_pole_green(E + d, c, Om, td, beta)).max())
    assert errs[-1] < 5e-5
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.6 < e0 / e1 < 4.4, errs


def test_dyson_tau_on_upm_mesh_agrees_with_matsubara_route():
    """Sigma^c of two fermionic poles given on a UPM mesh (splined onto the dense grid): the tau route
    and the i w route (Sigma^c(i w) by the spline-Filon transform, G = 1 / (i w - E - Sigma^c),
    truncated inverse transform with the reference term) both approach the closed form as the points
    per sub-interval double (m = 4, 8, 16): the tau route at second order in the dense spacing, the
    i w route faster; their difference shrinks with the tau route's error.  The tau route keeps
    G(0+) + G(beta-) = -1 to rounding."""
    beta = 16.0
    E, d = -0.2, 0.05
    poles = [(0.05, 0.5), (0.03, -0.7)]
    # closed form: the poles of 1 / (z - E - d - sum_a c_a / (z - w_a)) and their residues
    num = np.poly1d([1.0, -(E + d)])
    dens = [np.poly1d([1.0, -w]) for _, w in poles]
    poly = num * dens[0] * dens[1] - poles[0][0] * dens[1] - poles[1][0] * dens[0]
    z = np.roots(poly.coeffs).real
    res = [np.prod([zz - w for _, w in poles]) / np.prod([zz - y for y in z if y != zz]) for zz in z]
    et, en, diffs = [], [], []
    for m in (4, 8, 16):
        t = gi.upm_mesh(beta, 2 * m * 3, m)
        sig = sum(c * o.green0_tau(w, t, beta) for c, w in poles)
        td, Gd, Gm = o.dyson_tau(E, d, sig, t, beta)
        wn = o.matsubara(o.FERMION, 4096, beta)
        sig_iw = o.tau_to_iw(sig, t, beta, o.FERMION, 4096)
        Gn = o.iw_to_tau_fermion(1.0 / (1j * wn - (E + d) - sig_iw), t, beta, e_ref=np.float64(E + d))
        ex = sum(r * o.green0_tau(zz, t, beta) for r, zz in zip(res, z))
        et.append(np.abs(Gm - ex).max())
        en.append(np.abs(Gn - ex).max())
        diffs.append(np.abs(Gm - Gn).max())
        assert abs(Gd[0] + Gd[-1] + 1.0) < 1e-13
    for a, b in zip(et, et[1:]):
        assert 3.0 < a / b < 4.5, et
    for a, b in zip(en, en[1:]):
        assert a / b > 8.0, en
    assert diffs[-1] < 3e-4 and diffs[0] / diffs[-1] > 10.0, diffs


def _mutant_dyson_tau(E, dsig, sigc_tau, tau, beta):
    """dyson_tau with the jump at the integration end nodes read as the mean of the limits."""
    td = o.dense_grid(tau, beta)
    n = td.size
    dt = o.trapezoid_increments(td)
    g0 = lambda x: o.green0_tau(E, np.ravel(x), beta).reshape(np.shape(x))  # noqa: E731
    sc_d = o.spline_eval(tau, sigc_tau, td)
    sc = lambda x: np.interp(x, td, sc_d)  # noqa: E731
    G0c = o.fermion_kernel(g0, td, beta, "cols")
    Scr = o.fermion_kernel(sc, td, beta, "rows")
    for K in (G0c, Scr):
        K[0, 0] = K[n - 1, n - 1] = K[1, 1]
    Z = G0c * dsig + G0c @ (dt[:, None] * Scr)
    return td, np.linalg.solve(np.eye(n) - Z * dt[None, :], g0(td))


def test_planted_dyson_tau_end_node_mistake_is_caught():
    beta, E, d = 8.0, 0.3, -0.5
    errs = []
    for n in (32, 64):
        t = np.linspace(0, beta, n + 1)
        td, G = _mutant_dyson_tau(E, d, np.zeros(n + 1), t, beta)
        errs.append(np.abs(G - o.green0_tau(E + d, td, beta)).max())
    assert errs[0] / errs[1] < 3.0, errs
