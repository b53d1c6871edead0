"""Analytic continuation of Sigma^c to the real axis by a Pade approximant, quasiparticle energies.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may use it.

The paper continues Sigma^c_j(k | i w_n) to Sigma^c_j(k | w + i eta) after the path (analytic
continuation subsection of Sec. III.B) by the continuous-pole expansion and, for comparison, by
the Pade approximation of Vidberg and Serene (J. Low Temp. Phys. 29, 179 (1977)); quasiparticle
energies are read off A(w) = -Im G(w) / pi.  Here the Pade route:

* the continued fraction C(z) = a_0 / (1 + a_1 (z - z_0) / (1 + a_2 (z - z_1) / (1 + ...))) that
  interpolates the points (z_i, u_i) = (i w_i, Sigma^c(i w_i)), i < n_pade, with the coefficients of
  the Vidberg-Serene recursion g_0(z_j) = u_j,
  g_p(z_j) = (g_{p-1}(z_{p-1}) - g_{p-1}(z_j)) / ((z_j - z_{p-1}) g_{p-1}(z_j)),  a_p = g_p(z_p);
* G(w) = 1 / (w - e0 - Sigma^c(w + i eta)) with e0 = eps + Sigma_static - mu (energies from mu);
* the quasiparticle energy: the root x of x = e0 + Re Sigma^c(x + i eta) that Newton's method reaches
  from x = e0 (the peak of A(w) for a weakly damped state), reported as E = x + mu;
* the gap E_(N+1) - E_(N) of the quasiparticle energies in ascending order.
"""
from __future__ import annotations

import numpy as np


def pade_coefficients(z, u):
    """Coefficients a_p of the continued fraction through (z_i, u_i), i < N (last axis).

    z: complex [N]; u: complex [..., N] (leading axes are independent data sets)."""
    z = np.asarray(z, dtype=np.complex128)
    g = np.array(u, dtype=np.complex128, copy=True)
    N = g.shape[-1]
    a = np.empty_like(g)
    a[..., 0] = g[..., 0]
    for p in range(1, N):
        prev = g[..., p - 1:p].copy()             # g_{p-1}(z_{p-1}) = a_{p-1}
        gj = g[..., p:]
        g[..., p:] = (prev - gj) / ((z[p:] - z[p - 1]) * gj)
        a[..., p] = g[..., p]
    return a


def pade_eval(z, a, w):
    """C(w) by nesting the fraction from its last level: t = 1 + a_n (w - z_{n-1}) / t, n = N-1..1,
    then C = a_0 / t.  z: [N]; a: [..., N]; w: complex [..., M] or scalar broadcastable to a[..., :1]."""
    z = np.asarray(z, dtype=np.complex128)
    a = np.asarray(a)
    w = np.asarray(w, dtype=np.complex128)
    N = a.shape[-1]
    t = np.ones(np.broadcast(a[..., :1], w).shape, dtype=np.complex128)
    for n in range(N - 1, 0, -1):
        t = 1.0 + a[..., n:n + 1] * (w - z[n - 1]) / t
    return a[..., 0:1] / t


def pade_eval_and_derivative(z, a, w):
    """C(w) and dC/dw by the same nesting, with t_n' = (a_n - (w - z_{n-1}) a_n t_{n+1}' / t_{n+1}) / t_{n+1}."""
    z = np.asarray(z, dtype=np.complex128)
    a = np.asarray(a)
    w = np.asarray(w, dtype=np.complex128)
    N = a.shape[-1]
    shape = np.broadcast(a[..., :1], w).shape
    t = np.ones(shape, dtype=np.complex128)
    dt = np.zeros(shape, dtype=np.complex128)
    for n in range(N - 1, 0, -1):
        an, d = a[..., n:n + 1], w - z[n - 1]
        t_new = 1.0 + an * d / t
        dt = an / t - an * d * dt / (t * t)
        t = t_new
    c = a[..., 0:1] / t
    return c, -a[..., 0:1] * dt / (t * t)


def matsubara_points(n_pade, beta):
    """z_i = i w_i = i (2 i + 1) pi / beta, i < n_pade."""
    return 1j * (2 * np.arange(n_pade) + 1) * np.pi / beta


def qp_energies(eps, nb, sig_static, sigc_iw, mu, beta, n_pade, eta, iters=100, tol=1e-12):
    """Quasiparticle energies E_nk = x + mu, x = e0 + Re C_nk(x + i eta) by Newton from x = e0.

    eps, sig_static: [nk, nbmax]; sigc_iw: complex [nk, nbmax, niw] (positive Matsubara axis).
    Returns (E [nk, nbmax] with NaN for n >= Nb_k, converged [nk, nbmax] bool)."""
    nk, nbmax = eps.shape
    z = matsubara_points(n_pade, beta)
    a = pade_coefficients(z, sigc_iw[..., :n_pade])          # [nk, nbmax, n_pade]
    e0 = eps + sig_static - mu
    x = e0.copy()
    done = np.zeros_like(x, dtype=bool)
    for _ in range(iters):
        c, dc = pade_eval_and_derivative(z, a, (x + 1j * eta)[..., None])
        f = x - e0 - c[..., 0].real
        df = 1.0 - dc[..., 0].real
        step = f / df
        x = np.where(done, x, x - step)
        done |= np.abs(step) <= tol * (1.0 + np.abs(x))
    mask = np.arange(nbmax)[None, :] < np.asarray(nb)[:, None]
    return np.where(mask, x + mu, np.nan), done | ~mask


def spectral(eps, sig_static, sigc_iw, mu, beta, n_pade, eta, omega):
    """A_nk(w) = -(1/pi) Im 1 / (w - e0 - C_nk(w + i eta)) on the real grid omega (energies from mu)."""
    z = matsubara_points(n_pade, beta)
    a = pade_coefficients(z, sigc_iw[..., :n_pade])
    e0 = eps + sig_static - mu
    w = np.asarray(omega, dtype=np.float64)
    c = pade_eval(z, a, w[None, None, :] + 1j * eta)
    return -np.imag(1.0 / (w[None, None, :] + 1j * eta - e0[..., None] - c)) / np.pi


def qp_gap(E, nb, n_index):
    """E_(N+1) - E_(N) over the states n < Nb_k in ascending order (N = n_index, 1-based)."""
    mask = np.arange(E.shape[1])[None, :] < np.asarray(nb)[:, None]
    e = np.sort(E[mask])
    return float(e[n_index] - e[n_index - 1])


# ---------------------------------------------------------------------------
# continuous-pole expansion (CPE)
# ---------------------------------------------------------------------------
# The paper's own continuation (after Staar et al.): Im Sigma(w + i0) <= 0 (causality) is expanded in
# piecewise-linear functions of w with coefficients a_l >= 0, so that
#     Sigma(z) = (1/pi) int dw Im Sigma(w) / (w - z) = -(1/pi) sum_l a_l Phi_l(z),
#     Phi_l(z) = int dw h_l(w) / (w - z)                     (h_l: hat function at grid point w_l),
# and the a_l minimise the squared misfit to Sigma(i w_n) over the positive Matsubara points under
# a_l >= 0.  Readings: the hats sit at the interior points of a uniform real grid on [w_min, w_max]
# (Im Sigma vanishes at both ends); the spectral prefactor is 1/pi (the one that reproduces a pole
# r / (z - p) from Im Sigma = -pi r delta(w - p)); a ridge term ridge * max_l (B^T B)_ll * |a|^2 makes
# the non-negative least-squares problem strictly convex, so that its minimiser is unique.

def cpe_grid(w_min, w_max, n_real):
    """Uniform real grid w_0 .. w_{n_real-1}; the hats sit at w_1 .. w_{n_real-2}."""
    return np.linspace(float(w_min), float(w_max), int(n_real))


def cpe_phi(wgrid, z, derivative=False):
    """Phi_l(z) for the interior hats (last axis, n_real - 2), z complex (Im z > 0) broadcast in front.

    With F(a, b, c) = int_a^b (w - c) / (w - z) dw = (b - a) + (z - c) [ln(b - z) - ln(a - z)]:
    Phi_l = [F(w_{l-1}, w_l, w_{l-1}) - F(w_l, w_{l+1}, w_{l+1})] / (w_l - w_{l-1})."""
    w = np.asarray(wgrid, dtype=np.float64)
    z = np.asarray(z, dtype=np.complex128)[..., None]
    lo, mid, hi = w[:-2], w[1:-1], w[2:]
    dw = mid - lo

    def F(a, b, c):
        L = np.log(b - z) - np.log(a - z)
        val = (b - a) + (z - c) * L
        if not derivative:
            return val, None
        return val, L + (z - c) * (1.0 / (a - z) - 1.0 / (b - z))

    f1, d1 = F(lo, mid, lo)
    f2, d2 = F(mid, hi, hi)
    phi = (f1 - f2) / dw
    return (phi, (d1 - d2) / dw) if derivative else phi


def cpe_basis(wgrid, beta, n_iw):
    """Real design matrix [2 n_iw, n_real - 2]: rows Re then Im of -Phi_l(i w_n) / pi."""
    z = matsubara_points(n_iw, beta)
    B = -cpe_phi(wgrid, z) / np.pi
    return np.concatenate([B.real, B.imag], axis=0)


def cpe_fit(wgrid, beta, sigc_iw, ridge):
    """a_l >= 0 minimising |B a - y|^2 + lam |a|^2, lam = ridge * max_l (B^T B)_ll, per state.

    sigc_iw: complex [..., n_iw]; returns [..., n_real - 2]."""
    from scipy.optimize import nnls
    y = np.asarray(sigc_iw)
    n_iw = y.shape[-1]
    B = cpe_basis(wgrid, beta, n_iw)
    lam = ridge * np.max(np.sum(B * B, axis=0))
    Baug = np.concatenate([B, np.sqrt(lam) * np.eye(B.shape[1])], axis=0)
    flat = y.reshape(-1, n_iw)
    out = np.empty((flat.shape[0], B.shape[1]))
    for s in range(flat.shape[0]):
        rhs = np.concatenate([flat[s].real, flat[s].imag, np.zeros(B.shape[1])])
        out[s] = nnls(Baug, rhs, maxiter=50 * B.shape[1])[0]
    return out.reshape(y.shape[:-1] + (B.shape[1],))


def cpe_sigma(wgrid, a, z, derivative=False):
    """Sigma(z) = -(1/pi) sum_l a_l Phi_l(z) (and dSigma/dz); a: [..., n_real - 2], z: [...] complex."""
    if derivative:
        phi, dphi = cpe_phi(wgrid, z, derivative=True)
        return -np.sum(a * phi, axis=-1) / np.pi, -np.sum(a * dphi, axis=-1) / np.pi
    return -np.sum(a * cpe_phi(wgrid, z), axis=-1) / np.pi


def qp_energies_cpe(eps, nb, sig_static, sigc_iw, mu, beta, wgrid, ridge, eta, iters=100, tol=1e-12):
    """Quasiparticle energies from the CPE continuation: x = e0 + Re Sigma(x + i eta) by Newton from
    x = e0 (eta > 0).  Returns (E [nk, nbmax] with NaN for n >= Nb_k, converged, coefficients)."""
    a = cpe_fit(wgrid, beta, sigc_iw, ridge)
    e0 = eps + sig_static - mu
    x = e0.copy()
    done = np.zeros_like(x, dtype=bool)
    for _ in range(iters):
        s, ds = cpe_sigma(wgrid, a, x + 1j * eta, derivative=True)
        step = (x - e0 - s.real) / (1.0 - ds.real)
        x = np.where(done, x, x - step)
        done |= np.abs(step) <= tol * (1.0 + np.abs(x))
    mask = np.arange(eps.shape[1])[None, :] < np.asarray(nb)[:, None]
    return np.where(mask, x + mu, np.nan), done | ~mask, a


def spectral_cpe(eps, sig_static, a, mu, wgrid, eta, omega):
    """A(w) = -(1/pi) Im 1 / (w + i eta - e0 - Sigma(w + i eta)) with the CPE coefficients a."""
    e0 = eps + sig_static - mu
    w = np.asarray(omega, dtype=np.float64)
    s = cpe_sigma(wgrid, a[..., None, :], w + 1j * eta)
    return -np.imag(1.0 / (w + 1j * eta - e0[..., None] - s)) / np.pi
