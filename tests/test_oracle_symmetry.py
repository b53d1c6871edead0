"""Pins of the irreducible-wedge reduction (Sec. III.C) in the oracle, on the cubic-symmetric inputs.

The reduction is exact: with M(Rk, Rq, RG) = M(k, q, G), an invariant v and invariant band energies,
the full Brillouin-zone sums of Sigma^c and Sigma^x equal the sums over the irreducible q regrouped
with their stars, and P(Rq) is P(q) with its basis indices permuted.  A planted slip (R k in place of
R^-1 k) fails, and the irreducible counts are those of a Gamma-centred n^3 grid under O_h.
"""
import numpy as np
import pytest

import gwinputs as gi
import oracle as o

CUB = gi.tiny(name="cub3", grid=(3, 3, 3), nocc=2, nemp=2, ni=27, ntau=12, beta=20.0, niw=8)


@pytest.fixture(scope="module")
def cub():
    cfg = CUB
    prob = gi.make_cubic_problem(cfg)
    gen = gi.CubicGenerator(cfg)
    G = o.green0(prob.eps, prob.nb, prob.tau, cfg.beta)
    stars = o.ibz_stars(gen.rot_k)
    return cfg, prob, gen, G, stars


def test_group_and_ibz_counts():
    grp = gi.cubic_group()
    assert grp.shape == (48, 3, 3)
    # closed under products, orthogonal, distinct
    keys = {R.tobytes() for R in grp}
    assert len(keys) == 48
    for A in grp[::7]:
        for B in grp[::5]:
            assert (A @ B).tobytes() in keys
        assert (A @ A.T == np.eye(3, dtype=np.int64)).all()
    # irreducible points of Gamma-centred n^3 grids under O_h: 4 (n = 3), 10 (n = 4, 5), 20 (n = 6)
    for n, want in ((3, 4), (4, 10), (5, 10), (6, 20)):
        cfg = gi.tiny(name="g", grid=(n, n, n), ni=7)
        stars = o.ibz_stars(gi.rotation_k_maps(cfg))
        assert len(stars) == want
        assert sum(len(s) for _, s in stars) == n ** 3


def test_basis_shells_are_closed():
    for ni in (27, 57, 123, 691):
        g = gi.basis_vectors(ni)
        keys = {tuple(x) for x in g}
        for R in gi.cubic_group():
            assert {tuple(x) for x in g @ R.T} == keys
    with pytest.raises(ValueError):
        gi.basis_vectors(700)


def test_polarization_of_rotated_q_is_permuted(cub):
    cfg, prob, gen, G, stars = cub
    q = stars[1][0]
    P = o.polarization(gen.q_blocks(q), G, prob.kmq[q], cfg.scale)
    for qp, r in stars[1][1]:
        Pp = o.polarization(gen.q_blocks(qp), G, prob.kmq[qp], cfg.scale)
        perm = gen.rot_g[r]                          # index of R G_I
        assert np.abs(Pp[:, perm][:, :, perm] - P).max() < 1e-12 * np.abs(P).max()


def _contribs(cfg, prob, gen, G, qs):
    sc, sx = {}, {}
    occ = -G[:, :, -1]
    for q in qs:
        Mq = gen.q_blocks(q)
        P = o.polarization(Mq, G, prob.kmq[q], cfg.scale)
        _, R = o.screen(o.tau_to_iw(P, prob.tau, cfg.beta, o.BOSON, cfg.niw_b), prob.v[q])
        Wt = o.wt_tau(R, P, prob.v[q], prob.tau, cfg.beta)
        sc[q] = o.sigma_c(Mq, G, prob.kmq[q], Wt, cfg.scale)
        sx[q] = o.sigma_x(Mq, occ, prob.kmq[q], prob.v[q], cfg.scale)
    return sc, sx


def test_ibz_sums_equal_the_full_zone(cub):
    cfg, prob, gen, G, stars = cub
    sc, sx = _contribs(cfg, prob, gen, G, range(cfg.nk))
    full_c = sum(sc[q] for q in range(cfg.nk))
    full_x = sum(sx[q] for q in range(cfg.nk))
    ibz = [q for q, _ in stars]
    red_c = o.symmetrize_over_stars({q: sc[q] for q in ibz}, stars, gen.rot_k)
    red_x = o.symmetrize_over_stars({q: sx[q] for q in ibz}, stars, gen.rot_k)
    assert np.abs(red_c - full_c).max() < 1e-12 * np.abs(full_c).max()
    assert np.abs(red_x - full_x).max() < 1e-12 * np.abs(full_x).max()
    # the self-energy of a state depends on |k| only through the invariant energies: Sigma(R k) = Sigma(k)
    for r in (5, 17, 40):
        assert np.abs(full_c[gen.rot_k[r]] - full_c).max() < 1e-12 * np.abs(full_c).max()


def _mutant_symmetrize(contrib, stars, rot_k, kind):
    """symmetrize_over_stars with one planted mistake: 'weights' (each irreducible q counted |star|
    times at the same k, the shortcut that holds only for k-summed quantities) or 'forward' (R k in
    place of R^-1 k)."""
    total = 0
    for q, star in stars:
        for qp, r in star:
            C = contrib[q]
            total = total + (C if kind == "weights" else C[rot_k[r]])
    return total


@pytest.mark.parametrize("kind", ["weights", "forward"])
def test_planted_star_mistakes_are_caught(cub, kind):
    cfg, prob, gen, G, stars = cub
    ibz = [q for q, _ in stars]
    sc, _ = _contribs(cfg, prob, gen, G, range(cfg.nk))
    full_c = sum(sc[q] for q in range(cfg.nk))
    bad = _mutant_symmetrize({q: sc[q] for q in ibz}, stars, gen.rot_k, kind)
    assert np.abs(bad - full_c).max() > 1e-3 * np.abs(full_c).max()
