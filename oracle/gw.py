"""Plain FP64 implementation of one Matsubara-time GW pass.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions (readings of the paper; each is also listed in the design notes):

* Band index n is a band at k, m a band at k - q.  M^I_nm(k, q) is the
  paper's M^{k-q}_{mn}(G_I, q) (matrix-element equation, eq. mmatrix).
* s = -1 / (Omega N_k).  Since G(-tau) = -G(beta - tau) (Basics of the
  Theory), the polarization of eq. irpol becomes
  P_IJ(q,tau) = s sum_k sum_nm M^I_nm G_n(k,tau) G_m(k-q,beta-tau) conj(M^J_nm).
* tau[0] holds the 0+ limit and tau[-1] the beta- limit; the mesh must be
  mirror symmetric so that beta - tau_i is again a mesh point.
* The screened interaction is solved on the bosonic Matsubara axis
  (nu_n = 2 n pi / beta), where the W-tilde Dyson equation of the
  "Screened Coulomb potential" subsection is algebraic:
  W~ = v P v + v P W~  =>  W~ = v^1/2 [(1 - v^1/2 P v^1/2)^-1 - 1] v^1/2.
* The G Dyson equation (eqs. dysongf, zxjk, zcjk) is solved on the fermionic
  axis, G(i w) = 1 / (i w - E - Sigma^c(i w)), E = eps + Sigma_static - mu.
* Forward transforms follow eq. trans with a not-a-knot cubic spline of the
  tau data integrated exactly against e^{i w tau} ("Analytic continuation":
  cubic spline interpolation of the UPM grid).  Inverse transforms are
  truncated Matsubara sums plus reference terms known exactly in tau.
"""
from __future__ import annotations

import math

import numpy as np

FERMION = 0
BOSON = 1


# ---------------------------------------------------------------------------
# occupation and reference Green's function
# ---------------------------------------------------------------------------
def fermi(E, beta):
    """n_F(E) = 1 / (exp(beta E) + 1), evaluated without overflow."""
    E = np.asarray(E, dtype=np.float64)
    x = beta * E
    ex = np.exp(-np.abs(x))
    return np.where(x >= 0, ex / (1.0 + ex), 1.0 / (1.0 + ex))


def green0_tau(E, tau, beta):
    """Reference Green's function on the tau mesh.

    Paper, eq. for G^0 in "Green's function in the reference K-S system":
    G0(tau) = -exp(-E tau) [1 - n_F(E)], 0 <= tau <= beta.  Written as
    -exp(-E tau)/(1 + exp(-beta E)) for E >= 0 and
    -exp(E (beta - tau))/(1 + exp(beta E)) for E < 0 (algebraically equal).
    E: any shape; returns E.shape + (ntau,).
    """
    E = np.asarray(E, dtype=np.float64)[..., None]
    t = np.asarray(tau, dtype=np.float64)
    pos = -np.exp(-np.abs(E) * t) / (1.0 + np.exp(-beta * np.abs(E)))
    neg = -np.exp(-np.abs(E) * (beta - t)) / (1.0 + np.exp(-beta * np.abs(E)))
    return np.where(E >= 0, pos, neg)


def green0(eps, nb, tau, beta, mu=0.0):
    """G0_n(k, tau) for all (k, n < Nb_k) -> f64 [nk, nbmax, ntau] (zeros beyond Nb_k)."""
    G = green0_tau(eps - mu, tau, beta)
    mask = np.arange(eps.shape[1])[None, :] < np.asarray(nb)[:, None]
    return np.where(mask[..., None], G, 0.0)


# ---------------------------------------------------------------------------
# polarization (eq. irpol)
# ---------------------------------------------------------------------------
def polarization(Mq, G, kmq_q, s, taus=None, rows=None, cols=None):
    """P_IJ(q, tau_i) for one q.

    Mq: list over k of arrays [NI, Nb_k, Nb_{k-q}] (complex).
    G: [nk, nbmax, ntau] real.  kmq_q[k] = index of k - q.
    taus / rows / cols: optional index subsets of tau, I and J.
    Returns complex [len(taus), len(rows), len(cols)].
    """
    ntau = G.shape[2]
    taus = np.arange(ntau) if taus is None else np.asarray(taus)
    NI = Mq[0].shape[0]
    rows = np.arange(NI) if rows is None else np.asarray(rows)
    cols = np.arange(NI) if cols is None else np.asarray(cols)
    P = np.zeros((len(taus), len(rows), len(cols)), dtype=np.complex128)
    for k, Mk in enumerate(Mq):
        nn, nm = Mk.shape[1], Mk.shape[2]
        kq = int(kmq_q[k])
        A = Mk.reshape(NI, nn * nm)
        Ar, Ac = A[rows], A[cols]
        for a, i in enumerate(taus):
            # G_n(k, tau_i) G_m(k-q, beta - tau_i); beta - tau_i = tau_{N-i}
            g = np.outer(G[k, :nn, i], G[kq, :nm, ntau - 1 - i]).reshape(-1)
            P[a] += (Ar * g[None, :]) @ Ac.conj().T
    return s * P


# ---------------------------------------------------------------------------
# cubic spline and the tau -> i omega transform (eq. trans)
# ---------------------------------------------------------------------------
def spline_not_a_knot(tau, f):
    """Not-a-knot cubic spline through (tau_i, f_i) along axis 0.

    Returns (a, b, c, d), each [N, ...] for the N intervals, with
    S(tau_i + t) = a_i + b_i t + c_i t^2 + d_i t^3.
    """
    tau = np.asarray(tau, dtype=np.float64)
    n = tau.size
    if n < 4:
        raise ValueError("not-a-knot spline needs at least 4 points")
    f = np.asarray(f)
    h = np.diff(tau)
    # unknowns: second derivatives s_0..s_{n-1}
    A = np.zeros((n, n))
    rhs_shape = (n,) + f.shape[1:]
    R = np.zeros(rhs_shape, dtype=f.dtype if np.iscomplexobj(f) else np.float64)
    # not-a-knot at tau_1: third derivative continuous
    A[0, 0], A[0, 1], A[0, 2] = -1.0 / h[0], 1.0 / h[0] + 1.0 / h[1], -1.0 / h[1]
    for i in range(1, n - 1):
        A[i, i - 1] = h[i - 1]
        A[i, i] = 2.0 * (h[i - 1] + h[i])
        A[i, i + 1] = h[i]
        R[i] = 6.0 * ((f[i + 1] - f[i]) / h[i] - (f[i] - f[i - 1]) / h[i - 1])
    A[n - 1, n - 3] = -1.0 / h[n - 3]
    A[n - 1, n - 2] = 1.0 / h[n - 3] + 1.0 / h[n - 2]
    A[n - 1, n - 1] = -1.0 / h[n - 2]
    sig = np.linalg.solve(A, R.reshape(n, -1)).reshape(rhs_shape)
    hb = h.reshape((n - 1,) + (1,) * (f.ndim - 1))
    a = f[:-1]
    b = (f[1:] - f[:-1]) / hb - hb * (2.0 * sig[:-1] + sig[1:]) / 6.0
    c = sig[:-1] / 2.0
    d = (sig[1:] - sig[:-1]) / (6.0 * hb)
    return a, b, c, d


def filon_moments(w, h):
    """J_p(w, h) = int_0^h t^p e^{i w t} dt for p = 0..3 -> complex [len(w), len(h), 4].

    |w h| >= 0.5: J_0 = (e^{iwh} - 1)/(iw), J_p = (h^p e^{iwh} - p J_{p-1})/(iw).
    |w h| < 0.5: power series J_p = sum_j (iw)^j h^{p+j+1} / (j! (p+j+1)).
    """
    w = np.asarray(w, dtype=np.float64)[:, None]
    h = np.asarray(h, dtype=np.float64)[None, :]
    w, h = np.broadcast_arrays(w, h)
    J = np.zeros(w.shape + (4,), dtype=np.complex128)
    small = np.abs(w * h) < 0.5
    # series
    iw = 1j * w
    for p in range(4):
        acc = np.zeros(w.shape, dtype=np.complex128)
        term = np.ones(w.shape, dtype=np.complex128)  # (iw h)^j / j!
        for j in range(30):
            if j > 0:
                term = term * (iw * h) / j
            acc = acc + term / (p + j + 1)
        J[..., p] = np.where(small, acc * h ** (p + 1), 0.0)
    # recurrence
    big = ~small
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.exp(1j * w * h)
        prev = (e - 1.0) / iw
        J[..., 0] = np.where(big, prev, J[..., 0])
        for p in range(1, 4):
            cur = (h ** p * e - p * prev) / iw
            J[..., p] = np.where(big, cur, J[..., p])
            prev = cur
    return J


def matsubara(stat, n, beta):
    """omega_n = (2n+1) pi / beta (FERMION) or nu_n = 2 n pi / beta (BOSON)."""
    n = np.arange(n, dtype=np.float64)
    return (2.0 * n + 1.0) * math.pi / beta if stat == FERMION else 2.0 * n * math.pi / beta


def tau_to_iw(f, tau, beta, stat, niw, e_ref=None):
    """F(i w_n) = int_0^beta e^{i w_n tau} f(tau) dtau (eq. trans), tau on axis 0.

    f: [ntau, ...] real or complex.  The integrand is the not-a-knot cubic
    spline of f integrated exactly.  For FERMION with reference energies e_ref
    (shape f.shape[1:]) the spline is applied to f - G0(e_ref) and the exact
    transform 1/(i w - e_ref) of the reference is added back.
    Returns complex [niw, ...].
    """
    tau = np.asarray(tau, dtype=np.float64)
    f = np.asarray(f)
    w = matsubara(stat, niw, beta)
    if e_ref is not None:
        if stat != FERMION:
            raise ValueError("reference subtraction is for fermionic data")
        gref = np.moveaxis(green0_tau(e_ref, tau, beta), -1, 0)
        f = f - gref
    a, b, c, d = spline_not_a_knot(tau, f)
    J = filon_moments(w, np.diff(tau))                      # [niw, N, 4]
    ph = np.exp(1j * np.outer(w, tau[:-1]))                 # [niw, N]
    coef = np.stack([a, b, c, d], axis=-1)                  # [N, ..., 4]
    coef = np.moveaxis(coef, -1, 1)                         # [N, 4, ...]
    K = ph[:, :, None] * J                                  # [niw, N, 4]
    out = np.tensordot(K, coef, axes=([1, 2], [0, 1]))      # [niw, ...]
    if e_ref is not None:
        e = np.asarray(e_ref, dtype=np.float64)
        shape = (niw,) + (1,) * e.ndim
        out = out + 1.0 / (1j * w.reshape(shape) - e[None])
    return out


def iw_to_tau_fermion(F, tau, beta, e_ref=None):
    """f(tau_i) = G0(e_ref, tau_i) + (2/beta) sum_{n<niw} Re[e^{-i w_n tau_i} (F - 1/(i w_n - e_ref))].

    Inverse of eq. trans for a real fermionic function (F(-i w) = conj F(i w)),
    truncated at niw frequencies; the reference term carries the 0/beta jump.
    F: [niw, ...] complex.  Returns real [ntau, ...].
    """
    F = np.asarray(F)
    niw = F.shape[0]
    w = matsubara(FERMION, niw, beta)
    shape = (niw,) + (1,) * (F.ndim - 1)
    D = F
    if e_ref is not None:
        D = F - 1.0 / (1j * w.reshape(shape) - np.asarray(e_ref)[None])
    ph = np.exp(-1j * np.outer(tau, w))                     # [ntau, niw]
    out = (2.0 / beta) * np.real(np.tensordot(ph, D, axes=([1], [0])))
    if e_ref is not None:
        out = out + np.moveaxis(green0_tau(e_ref, tau, beta), -1, 0)
    return out


def iw_to_tau_boson_herm(R, tau, beta, add_tau=None):
    """f(tau_i) = add(tau_i) + (1/beta)[R_0 + sum_{n>=1}(e^{-i nu_n tau_i} R_n + e^{i nu_n tau_i} R_n^H)].

    Inverse bosonic transform of matrices with R(-i nu) = R(i nu)^H, which
    holds for the screened interaction because P(tau) is Hermitian.
    R: [niw, n, n].  Returns complex [ntau, n, n].
    """
    R = np.asarray(R)
    niw = R.shape[0]
    nu = matsubara(BOSON, niw, beta)
    ph = np.exp(-1j * np.outer(tau, nu))                    # [ntau, niw]
    RH = np.conj(np.swapaxes(R, 1, 2))
    out = np.tensordot(ph[:, 1:], R[1:], axes=([1], [0])) \
        + np.tensordot(np.conj(ph[:, 1:]), RH[1:], axes=([1], [0]))
    out = (out + R[0][None]) / beta
    if add_tau is not None:
        out = out + add_tau
    return out


# ---------------------------------------------------------------------------
# screened interaction on the nu axis
# ---------------------------------------------------------------------------
def screen(P_iw, v):
    """W~(q, i nu) from P(q, i nu) for one q.

    chi~ = v^1/2 P v^1/2; solve (1 - chi~) X = chi~ (LU with partial
    pivoting); W~ = v^1/2 X v^1/2; R = W~ - v P v.
    This is the W-tilde Dyson equation of the screened-interaction subsection
    (W~ = v P v + v P W~) after the tau convolution becomes a product on the
    Matsubara axis.  P_iw: [niw, NI, NI]; v: [NI].  Returns (W~, R).
    """
    sv = np.sqrt(np.asarray(v, dtype=np.float64))
    n = sv.size
    W = np.empty_like(P_iw, dtype=np.complex128)
    for i in range(P_iw.shape[0]):
        chi = sv[:, None] * P_iw[i] * sv[None, :]
        X = np.linalg.solve(np.eye(n) - chi, chi)
        W[i] = sv[:, None] * X * sv[None, :]
    vPv = np.asarray(v)[None, :, None] * P_iw * np.asarray(v)[None, None, :]
    return W, W - vPv


def wt_tau(R_iw, P_tau, v, tau, beta):
    """W~(q, tau) = v P(q, tau) v + inverse transform of R = W~ - v P v."""
    v = np.asarray(v)
    vPv = v[None, :, None] * P_tau * v[None, None, :]
    return iw_to_tau_boson_herm(R_iw, tau, beta, add_tau=vPv)


# ---------------------------------------------------------------------------
# self-energy (eq. sigc) and exchange (product-basis form of eq. sigx)
# ---------------------------------------------------------------------------
def sigma_c(Mq, G, kmq_q, Wt_tau, s, full=False, taus=None, ks=None):
    """Contribution of one q to the correlation self-energy.

    Eq. sigc: Sigma^c_n(k, tau) = s sum_q sum_m G_m(k-q, tau)
    sum_IJ conj(M^I_nm) W~_IJ(q, tau) M^J_nm.
    DIAG (full=False): returns real [len(ks), nbmax, len(taus)].
    FULL: returns complex [len(ks), nbmax, nbmax, len(taus)] with
    Sigma_nn' = s sum_m G_m sum_IJ conj(M^I_nm) W~_IJ M^J_n'm.
    """
    nk = len(Mq)
    ntau = G.shape[2]
    taus = np.arange(ntau) if taus is None else np.asarray(taus)
    ks = np.arange(nk) if ks is None else np.asarray(ks)
    nbmax = G.shape[1]
    if full:
        out = np.zeros((len(ks), nbmax, nbmax, len(taus)), dtype=np.complex128)
    else:
        out = np.zeros((len(ks), nbmax, len(taus)), dtype=np.float64)
    for a, k in enumerate(ks):
        Mk = Mq[k]
        NI, nn, nm = Mk.shape
        kq = int(kmq_q[k])
        A = Mk.reshape(NI, nn * nm)
        for b, i in enumerate(taus):
            Y = Wt_tau[i] @ A                                   # [NI, nn*nm]
            gm = G[kq, :nm, i]
            if full:
                Y3 = Y.reshape(NI, nn, nm)
                # sum_m g_m sum_I conj(M^I_nm) Y^I_n'm
                out[a, :nn, :nn, b] += s * np.einsum("inm,ipm,m->np", Mk.conj(), Y3, gm)
            else:
                sig = np.sum(A.conj() * Y, axis=0).reshape(nn, nm)
                scale = np.max(np.abs(sig)) if sig.size else 0.0
                if scale > 0 and np.max(np.abs(sig.imag)) > 1e-9 * scale:
                    raise AssertionError("quadratic form of W~ not real: W~ not Hermitian")
                out[a, :nn, b] += s * (sig.real @ gm)
    return out


def sigma_x(Mq, occ, kmq_q, v, s, full=False):
    """Contribution of one q to the exchange self-energy.

    Sigma^x = -G(tau -> 0-) v delta(tau) ("Screened Coulomb potential" and
    eq. sigx with f = G(0-)); in the product basis
    Sigma^x_nn'(k) = s sum_q sum_m f_m(k-q) sum_I v_I conj(M^I_nm) M^I_n'm.
    occ: [nk, nbmax] occupations f = -G(beta-).
    """
    nk = len(Mq)
    nbmax = occ.shape[1]
    v = np.asarray(v)
    out = np.zeros((nk, nbmax, nbmax) if full else (nk, nbmax),
                   dtype=np.complex128 if full else np.float64)
    for k, Mk in enumerate(Mq):
        NI, nn, nm = Mk.shape
        f = occ[int(kmq_q[k]), :nm]
        if full:
            out[k, :nn, :nn] += s * np.einsum("i,inm,ipm,m->np", v, Mk.conj(), Mk, f)
        else:
            out[k, :nn] += s * np.einsum("i,inm,m->n", v, np.abs(Mk) ** 2, f)
    return out


# ---------------------------------------------------------------------------
# Dyson equation for G and the chemical potential
# ---------------------------------------------------------------------------
def dyson_G_iw(E, sigc_iw, beta):
    """G(i w_n) = 1 / (i w_n - E - Sigma^c(i w_n)); E, sigc_iw [nk, nb] / [nk, nb, niw]."""
    w = matsubara(FERMION, sigc_iw.shape[-1], beta)
    return 1.0 / (1j * w[None, None, :] - E[..., None] - sigc_iw)


def particle_number(E, sigc_iw, beta, mask):
    """N = sum_nk [n_F(E) + (2/beta) sum_n Re(G - G_ref)(i w_n)], G_ref = 1/(i w - E).

    This is N = -sum G(beta-) (occupations f = G(0-) of eq. sigx, with
    G(0-) = -G(beta-)) evaluated from the truncated Matsubara sum.
    """
    w = matsubara(FERMION, sigc_iw.shape[-1], beta)
    G = dyson_G_iw(E, sigc_iw, beta)
    Gr = 1.0 / (1j * w[None, None, :] - E[..., None])
    per = fermi(E, beta) + (2.0 / beta) * np.sum((G - Gr).real, axis=-1)
    return float(np.sum(np.where(mask, per, 0.0)))


def dyson(eps, nb, sig_static, sigc_iw, beta, tau, n_target, mu0=0.0,
          search=True, nsteps=200):
    """Dyson update of the diagonal G and the chemical potential.

    E(mu) = eps + Sigma_static - mu.  mu by bisection on
    [min E - 50/beta, max E + 50/beta] (fixed number of halvings) so that
    N(mu) = n_target.  Returns dict(mu, N, G_iw, G_tau, E).
    """
    mask = np.arange(eps.shape[1])[None, :] < np.asarray(nb)[:, None]
    E0 = np.where(mask, eps + sig_static, 0.0)
    sig = np.where(mask[..., None], sigc_iw, 0.0)
    if search:
        lo = float(E0[mask].min()) - 50.0 / beta
        hi = float(E0[mask].max()) + 50.0 / beta
        for _ in range(nsteps):
            mid = 0.5 * (lo + hi)
            if particle_number(E0 - mid, sig, beta, mask) < n_target:
                lo = mid
            else:
                hi = mid
        mu = 0.5 * (lo + hi)
    else:
        mu = mu0
    E = E0 - mu
    G_iw = np.where(mask[..., None], dyson_G_iw(E, sig, beta), 0.0)
    G_tau = iw_to_tau_fermion(np.moveaxis(G_iw, -1, 0), tau, beta, e_ref=E)
    G_tau = np.where(mask[..., None], np.moveaxis(G_tau, 0, -1), 0.0)
    N = particle_number(E, sig, beta, mask)
    return dict(mu=mu, N=N, G_iw=G_iw, G_tau=G_tau, E=E)


# ---------------------------------------------------------------------------
# crystal symmetry: q in the irreducible wedge (Sec. III.C)
# ---------------------------------------------------------------------------
def ibz_stars(rot_k):
    """The irreducible q points and their stars under a point group given by its action on the k grid
    (rot_k[r, k] = index of R_r k): every orbit {R q} is represented by its smallest index, and its star
    lists each member q' once with the first operation r (in the given order) that maps the
    representative onto it.  Returns [(q_ibz, [(q', r), ...]), ...] in increasing q_ibz."""
    rot_k = np.asarray(rot_k)
    nk = rot_k.shape[1]
    seen = np.zeros(nk, dtype=bool)
    out = []
    for q in range(nk):
        if seen[q]:
            continue
        star = []
        for r in range(rot_k.shape[0]):
            qp = int(rot_k[r, q])
            if not seen[qp]:
                seen[qp] = True
                star.append((qp, r))
        out.append((q, star))
    return out


def symmetrize_over_stars(contrib, stars, rot_k):
    """The paper's regrouping of the self-energy's q sum over the irreducible wedge (the equation that
    follows the relations for M, P and W~ in Sec. III.C): the contribution of q' = R q to state (k, n)
    equals that of q to (R^-1 k, n), so

        S_n(k) = sum_{q in IBZ} sum_{(q', R) in star(q)} C_q,n(R^-1 k),

    contrib: {q_ibz: C_q [nk, ...]} (the contributions of each irreducible q to every k, e.g. sigma_c
    or sigma_x of that q).  Returns the sum [nk, ...]."""
    rot_k = np.asarray(rot_k)
    nk = rot_k.shape[1]
    total = None
    for q, star in stars:
        C = np.asarray(contrib[q])
        for qp, r in star:
            inv = np.empty(nk, dtype=np.int64)
            inv[rot_k[r]] = np.arange(nk)          # inv[k] = R^-1 k
            term = C[inv]
            total = term if total is None else total + term
    return total


# ---------------------------------------------------------------------------
# the paper's own tau-domain solvers (cross-checks of the Matsubara-axis forms)
# ---------------------------------------------------------------------------
def spline_eval(tau, f, x):
    """The not-a-knot cubic spline of f (mesh tau, axis 0) evaluated at points x in [tau_0, tau_N]."""
    tau = np.asarray(tau, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    a, b, c, d = spline_not_a_knot(tau, f)
    i = np.clip(np.searchsorted(tau, x, side="right") - 1, 0, tau.size - 2)
    t = (x - tau[i]).reshape(x.shape + (1,) * (np.ndim(f) - 1))
    return a[i] + t * (b[i] + t * (c[i] + t * d[i]))


def trapezoid_increments(tau):
    """The paper's increments of the tau-domain linear systems: (tau_{i+1} - tau_{i-1}) / 2 inside,
    (tau_1 - tau_0) / 2 and (tau_M - tau_{M-1}) / 2 at the ends ("Screened Coulomb potential")."""
    tau = np.asarray(tau, dtype=np.float64)
    d = np.empty_like(tau)
    d[1:-1] = 0.5 * (tau[2:] - tau[:-2])
    d[0] = 0.5 * (tau[1] - tau[0])
    d[-1] = 0.5 * (tau[-1] - tau[-2])
    return d


def wt_tau_system(P_tau, v, tau, beta):
    """W~(q, tau) on the mesh from the paper's tau-domain linear system (eq. tildeW):

        sum_r [delta_pr 1 - A(tau_p - tau_r) dtau_r] W~(tau_r) = A(tau_p) v,   A = v P,

    with the trapezoid increments dtau_r.  A at tau_p - tau_r < 0 is taken at tau_p - tau_r + beta
    (bosonic periodicity of P), and between mesh points from the not-a-knot cubic spline of P(tau)
    (the reading of "discretise on the UPM grid": the differences of mesh points are not mesh points).
    P_tau: [ntau, NI, NI]; v: [NI].  One dense solve of order ntau * NI.  Returns [ntau, NI, NI].
    """
    tau = np.asarray(tau, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    N, NI = tau.size, v.size
    dt = trapezoid_increments(tau)
    x = tau[:, None] - tau[None, :]
    x = np.where(x < 0.0, x + beta, x)
    Px = spline_eval(tau, P_tau, x.reshape(-1)).reshape(N, N, NI, NI)
    A = v[None, None, :, None] * Px                             # v P(tau_p - tau_r)
    K = -A * dt[None, :, None, None]                           # [p, r, I, J]
    K = np.moveaxis(K, 1, 2).reshape(N * NI, N * NI).astype(np.complex128)   # rows (p, I), cols (r, J)
    K += np.eye(N * NI)
    rhs = v[None, :, None] * np.asarray(P_tau) * v[None, None, :]   # A(tau_p) v
    W = np.linalg.solve(K, rhs.reshape(N * NI, NI))
    return W.reshape(N, NI, NI)


def dense_grid(tau, beta):
    """The uniform grid of the tau-domain Dyson solve: spacing tau_1 - tau_0 (the smallest of a
    power mesh) from 0 to beta (eq. dysong)."""
    h = tau[1] - tau[0]
    n = int(round(beta / h))
    if abs(n * h - beta) > 1e-9 * beta:
        raise ValueError("beta is not a multiple of tau_1 - tau_0")
    return np.linspace(0.0, beta, n + 1)


def fermion_kernel(f_of, t, beta, integrate):
    """The matrix f(t_a - t_b) over a grid t of [0, beta] for a fermionic f known on [0, beta]
    (f(x) = -f(x + beta) for x < 0), as the integrand of a trapezoid sum over the columns
    (integrate="cols", the variable is t_b) or over the rows (integrate="rows", the variable is t_a).
    Where f jumps (x = 0) an interior node takes the mean of the two limits; an end node of the
    integration range takes the one limit inside the range: at t_a = t_b = 0 the variable lies above
    the other argument, at t_a = t_b = beta below it.
    """
    x = t[:, None] - t[None, :]
    pos = f_of(np.where(x > 0, x, 0.0))
    neg = -f_of(np.where(x < 0, x + beta, beta))
    f0p, f0m = f_of(np.zeros(1))[0], -f_of(np.full(1, beta))[0]      # f(0+), f(0-)
    out = np.where(x > 0, pos, neg)
    n = t.size - 1
    out[np.arange(n + 1), np.arange(n + 1)] = 0.5 * (f0p + f0m)
    if integrate == "cols":          # variable t_b: at 0 it is above t_a = 0 (x -> 0-), at beta below
        out[0, 0], out[n, n] = f0m, f0p
    else:                            # variable t_a: at 0 it is above t_b = 0 (x -> 0+), at beta below
        out[0, 0], out[n, n] = f0p, f0m
    return out


def dyson_tau(E, dsig, sigc_tau, tau, beta):
    """G_j(k, tau) of one state from the paper's tau-domain Dyson equation (eqs. dysongf, zxjk, zcjk,
    dysong): G = G0 + int_0^beta dt2 Z(t, t2) G(t2) with

        Z^x(t, t2) = G0(t - t2) dsig,    Z^c(t, t2) = int_0^beta dt1 G0(t - t1) Sigma^c(t1 - t2),

    solved as sum_r [delta_pr - dt_r Z(t_p, t_r)] G(t_r) = G0(t_p) on the dense uniform grid of
    spacing tau_1 - tau_0 onto which Sigma^c is splined (not-a-knot).  G0 is the reference Green's
    function at energy E (from mu), dsig = Sigma^x + Sigma^H - Sigma_0 the static difference; negative
    arguments use antiperiodicity, and the jumps at zero argument are taken as fermion_kernel states;
    both the t2 and the t1 integrals use the trapezoid increments of the dense grid.
    Returns (t_dense, G on t_dense, G at the mesh points tau).
    """
    td = dense_grid(tau, beta)
    n = td.size
    dt = trapezoid_increments(td)
    g0 = lambda x: green0_tau(E, np.ravel(x), beta).reshape(np.shape(x))  # noqa: E731
    sc_d = spline_eval(tau, sigc_tau, td)                       # Sigma^c on the dense grid
    sc = lambda x: np.interp(x, td, sc_d)                       # noqa: E731 (x on the grid)
    G0c = fermion_kernel(g0, td, beta, "cols")                 # G0(t_p - t_r), r integrated
    Scr = fermion_kernel(sc, td, beta, "rows")                 # Sigma^c(t_s - t_r), s integrated
    Zc = G0c @ (dt[:, None] * Scr)
    Z = G0c * dsig + Zc
    A = np.eye(n) - Z * dt[None, :]
    G = np.linalg.solve(A, g0(td))
    idx = np.rint(np.asarray(tau) / (td[1] - td[0])).astype(int)
    return td, G, G[idx]


def iw_to_tau_fermion_matrix(D, tau, beta):
    """(1/beta) sum_{n>=0} [e^{-i w_n tau} D_n + e^{+i w_n tau} D_n^H] for band matrices D_n.

    The inverse of eq. trans for a Hermitian-in-tau fermionic matrix function, whose negative
    frequencies are D(-i w) = D(i w)^H.  D: [..., nb, nb, niw] -> [..., nb, nb, ntau].
    """
    D = np.asarray(D)
    niw = D.shape[-1]
    w = matsubara(FERMION, niw, beta)
    ph = np.exp(-1j * np.outer(tau, w))                     # [ntau, niw]
    DH = np.conj(np.swapaxes(D, -3, -2))
    return (np.tensordot(D, ph.T, axes=([-1], [0])) + np.tensordot(DH, np.conj(ph).T, axes=([-1], [0]))) / beta


def static_bracket(H0, mask, beta):
    """Bracket of the chemical potential for band matrices: the Gershgorin discs of the static
    matrices H0 = eps + Sigma_static (each eigenvalue lies within sum_{i != j} |H0_ij| of some
    diagonal entry H0_jj), widened by 50 / beta on both sides."""
    lo, hi = np.inf, -np.inf
    for k in range(H0.shape[0]):
        n = int(mask[k].sum())
        A = H0[k, :n, :n]
        r = np.sum(np.abs(A), axis=1) - np.abs(np.diag(A))
        d = np.real(np.diag(A))
        lo, hi = min(lo, float(np.min(d - r))), max(hi, float(np.max(d + r)))
    return lo - 50.0 / beta, hi + 50.0 / beta


def dyson_matrix(eps, nb, sig_static, sigc_iw, beta, tau, n_target, mu0=0.0, search=True,
                 nsteps=200):
    """Dyson update of the full band-matrix G: the generalisation of the diagonal approximation to
    off-diagonal Sigma_nn' (eqs. dysongf, zxjk, zcjk with matrices, solved on the fermionic axis).

    H0(k) = diag(eps_k) + Sigma_static(k); G(k, i w) = [(i w + mu) 1 - H0(k) - Sigma^c(k, i w)]^-1
    over the bands n < Nb_k.  With the diagonal reference G_ref = diag(1 / (i w - E_jj)),
    E_jj = H0_jj - mu, and D = G - G_ref:
      G(tau) = diag(G0(E_jj, tau)) + inverse transform of D (negative frequencies D^H),
      N(mu) = sum_k [sum_j n_F(E_jj) + (2/beta) sum_n Re Tr D(i w_n)]  (= -sum_k Tr G(beta-)).
    mu by bisection on the Gershgorin bracket of H0 (static_bracket), as in the diagonal case.
    eps [nk, nbmax]; sig_static [nk, nbmax, nbmax]; sigc_iw [nk, nbmax, nbmax, niw].
    Returns dict(mu, N, G_iw [nk, nb, nb, niw], G_tau [nk, nb, nb, ntau]).
    """
    nk, nbmax = eps.shape
    niw = sigc_iw.shape[-1]
    w = matsubara(FERMION, niw, beta)
    mask = np.arange(nbmax)[None, :] < np.asarray(nb)[:, None]
    H0 = np.zeros((nk, nbmax, nbmax), dtype=np.complex128)
    for k in range(nk):
        n = int(nb[k])
        H0[k, :n, :n] = np.diag(eps[k, :n]) + sig_static[k, :n, :n]

    def green(mu):
        G = np.zeros((nk, nbmax, nbmax, niw), dtype=np.complex128)
        for k in range(nk):
            n = int(nb[k])
            for i in range(niw):
                A = (1j * w[i] + mu) * np.eye(n) - H0[k, :n, :n] - sigc_iw[k, :n, :n, i]
                G[k, :n, :n, i] = np.linalg.inv(A)
        return G

    def number(mu):
        G = green(mu)
        tot = 0.0
        for k in range(nk):
            n = int(nb[k])
            E = np.real(np.diag(H0[k, :n, :n])) - mu
            ref = 1.0 / (1j * w[None, :] - E[:, None])          # [n, niw]
            trD = np.trace(G[k, :n, :n, :], axis1=0, axis2=1) - ref.sum(axis=0)
            tot += float(np.sum(fermi(E, beta)) + (2.0 / beta) * np.sum(trD.real))
        return tot

    if search:
        lo, hi = static_bracket(H0, mask, beta)
        for _ in range(nsteps):
            mid = 0.5 * (lo + hi)
            if number(mid) < n_target:
                lo = mid
            else:
                hi = mid
        mu = 0.5 * (lo + hi)
    else:
        mu = mu0
    G_iw = green(mu)
    G_tau = np.zeros((nk, nbmax, nbmax, tau.size), dtype=np.complex128)
    for k in range(nk):
        n = int(nb[k])
        E = np.real(np.diag(H0[k, :n, :n])) - mu
        ref = 1.0 / (1j * w[None, :] - E[:, None])
        D = G_iw[k, :n, :n, :].copy()
        D[np.arange(n), np.arange(n), :] -= ref
        G_tau[k, :n, :n, :] = iw_to_tau_fermion_matrix(D, tau, beta)
        G_tau[k, np.arange(n), np.arange(n), :] += green0_tau(E, tau, beta)
    return dict(mu=mu, N=number(mu), G_iw=G_iw, G_tau=G_tau)


def gap_proxy(eps, nb, sig_static, sigc_iw0, mu, n_target):
    """Matsubara-axis gap proxy: E^QP = eps + Sigma_static + Re Sigma^c(i w_0) - mu,
    sorted over all (n, k); gap = E_(N+1) - E_(N) with N = round(n_target)."""
    mask = np.arange(eps.shape[1])[None, :] < np.asarray(nb)[:, None]
    e = (eps + sig_static + np.real(sigc_iw0) - mu)[mask]
    e = np.sort(e)
    N = int(round(n_target))
    return float(e[N] - e[N - 1])


# ---------------------------------------------------------------------------
# one pass / the self-consistent loop
# ---------------------------------------------------------------------------
def gw_pass(prob, Mgen, G, Wt_cache=None, full=False, keep=False):
    """One pass P -> W~ -> Sigma for all q (paper's self-consistent scheme).

    prob: gwinputs.Problem; Mgen: object with q_blocks(q); G: [nk, nbmax, ntau].
    Wt_cache: optional list of W~(q, tau) to reuse (GW0).
    Returns dict(sigc_tau, sigx, Wt) (and P_tau, P_iw per q when keep=True).
    """
    cfg = prob.cfg
    nk = cfg.nk
    s = cfg.scale
    tau = prob.tau
    nbmax = G.shape[1]
    sigc = np.zeros((nk, nbmax, nbmax, tau.size) if full else (nk, nbmax, tau.size),
                    dtype=np.complex128 if full else np.float64)
    occ = -G[:, :, -1]
    sigx = np.zeros((nk, nbmax, nbmax) if full else (nk, nbmax),
                    dtype=np.complex128 if full else np.float64)
    Wts, extra = [], []
    for q in range(nk):
        Mq = Mgen.q_blocks(q)
        if Wt_cache is None:
            P_tau = polarization(Mq, G, prob.kmq[q], s)
            P_iw = tau_to_iw(P_tau, tau, cfg.beta, BOSON, cfg.niw_b)
            _, R = screen(P_iw, prob.v[q])
            Wt = wt_tau(R, P_tau, prob.v[q], tau, cfg.beta)
            if keep:
                extra.append(dict(P_tau=P_tau, P_iw=P_iw, R_iw=R))
        else:
            Wt = Wt_cache[q]
        Wts.append(Wt)
        sigc += sigma_c(Mq, G, prob.kmq[q], Wt, s, full=full)
        sigx += sigma_x(Mq, occ, prob.kmq[q], prob.v[q], s, full=full)
    return dict(sigc_tau=sigc, sigx=sigx, Wt=Wts, extra=extra)


def run_loop(prob, Mgen, mode="g0w0", niter=1, v_ref=None):
    """G0W0 (first iteration only), GW0 (W~ frozen after iteration 1) or scGW.

    Loop structure of the "Scheme for scGW" subsection.  Returns a list of
    per-iteration dicts (sigc_tau, sigx, sigc_iw, mu, N, gap, G_tau).
    """
    cfg = prob.cfg
    tau = prob.tau
    mu = 0.0
    G = green0(prob.eps, prob.nb, tau, cfg.beta, mu)
    Wt = None
    hist = []
    for it in range(niter if mode != "g0w0" else 1):
        res = gw_pass(prob, Mgen, G, Wt_cache=Wt if mode == "gw0" else None)
        if mode == "gw0" and Wt is None:
            Wt = res["Wt"]
        sig_static = res["sigx"] - (0.0 if v_ref is None else v_ref)
        sigc_iw = np.moveaxis(tau_to_iw(np.moveaxis(res["sigc_tau"], -1, 0), tau,
                                        cfg.beta, FERMION, cfg.niw_f), 0, -1)
        rec = dict(sigc_tau=res["sigc_tau"], sigx=res["sigx"], sigc_iw=sigc_iw)
        if mode == "g0w0":
            rec.update(mu=mu, N=None, G_tau=G)
        else:
            d = dyson(prob.eps, prob.nb, sig_static, sigc_iw, cfg.beta, tau,
                      prob.n_target)
            G = d["G_tau"]
            mu = d["mu"]
            rec.update(mu=mu, N=d["N"], G_tau=G)
        rec["gap"] = gap_proxy(prob.eps, prob.nb, sig_static, sigc_iw[..., 0], mu,
                               prob.n_target)
        hist.append(rec)
    return hist
