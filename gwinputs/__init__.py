"""Seeded synthetic inputs for the Matsubara-time GW hot path.

This module is shared by the FP64 oracle (``oracle/``), the tests and the
benchmark.  It holds *inputs only*: k-grids, the imaginary-time mesh, model
band energies, the diagonal Coulomb kernel and the plane-wave matrix elements
M drawn from a counter-based generator.  None of the method's arithmetic
(G0, P, W, Sigma, transforms, Dyson) lives here.

What the inputs stand in for (the paper's workloads are all-electron LAPW
calculations of real crystals, which are not available here):

* k-mesh: Gamma-centred N1 x N2 x N3 grid, k_d = i_d / N_d; the q-grid equals
  the k-grid (the paper samples 4x4x4, and 6x6x6 for diamond; Computational
  Details section).
* tau mesh: uniform, or the uniform power mesh (UPM) of the "Matsubara-time
  sampling" subsection, built as: n intervals, m = 5 sub-points per power
  interval, p_h = n / (2m) power intervals on [0, beta/2] with nodes
  0, (beta/2) 2^(j - p_h) (j = 1..p_h), each split into m equal pieces, then
  mirrored onto [beta/2, beta].  n = 80 gives the paper's 81 points.
* energies: eps_nk = eps_n + 0.05 * sum_d cos(2 pi k_d) with eps_n on
  inclusive linspaces per band group (occupied groups first).
* v_I(q) = 4 pi / (0.1 + 0.09 I), I 0-based: a diagonal stand-in for the
  Coulomb kernel 4 pi / |q + G|^2 of the screened-interaction subsection.
* M^I_nm(k, q): complex Gaussian with E|M|^2 = 1 / (1 + I/16).  n is a band
  at k, m a band at k - q; in the paper's notation this is the element
  M^{k-q}_{mn}(G_I, q) of the matrix-element equation.  By default M obeys
  the time-reversal / pair symmetry of real matrix elements (a Klein group
  {e, a, b, ab}, with a: (k,q,n,m) -> (q-k,q,m,n) and
  b: (k,q,n,m) -> (-k,-q,n,m) plus complex conjugation), so that
  P(q,tau) = P(q,beta-tau) and P(q,i nu) is Hermitian.  One Gaussian is drawn
  per orbit, keyed by the orbit's smallest linear index; an orbit fixed by a
  conjugating element is real.

Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11) with Box-Muller in FP64, so the
device generator in the HIP library can reproduce the same integers from the
published definition.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Philox4x32-10 (published definition, SC'11) and Box-Muller in FP64
# ---------------------------------------------------------------------------
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85

# stream tags, placed in counter word 3, keep the draws of different inputs apart
TAG_M = 0x4D475731        # matrix elements M
TAG_NB = 0x4E42434E       # per-k band counts (uneven configuration)
TAG_NI = 0x4E49434E       # per-q product-basis sizes (uneven configuration)

_U32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, key):
    """Vectorised Philox4x32 with 10 rounds.

    c0..c3: uint32 arrays (broadcastable), key: python int (64-bit seed,
    split as k0 = low 32 bits, k1 = high 32 bits).  Returns four uint32 arrays.
    """
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.asarray(c1, dtype=np.uint64)
    c2 = np.asarray(c2, dtype=np.uint64)
    c3 = np.asarray(c3, dtype=np.uint64)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = int(key) & 0xFFFFFFFF
    k1 = (int(key) >> 32) & 0xFFFFFFFF
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    for _ in range(10):
        p0 = m0 * c0          # < 2^64, exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _U32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _U32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
        k0 = (k0 + PHILOX_W0) & 0xFFFFFFFF
        k1 = (k1 + PHILOX_W1) & 0xFFFFFFFF
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def uniform53(ra, rb):
    """Two uint32 words -> double in (0, 1): ((ra>>5)*2^26 + (rb>>6) + 0.5) / 2^53."""
    ra = np.asarray(ra, dtype=np.uint64) >> np.uint64(5)
    rb = np.asarray(rb, dtype=np.uint64) >> np.uint64(6)
    return (ra.astype(np.float64) * 67108864.0 + rb.astype(np.float64) + 0.5) \
        * (1.0 / 9007199254740992.0)


def box_muller(r0, r1, r2, r3):
    """Philox output -> two independent N(0,1) doubles (Box-Muller)."""
    u1 = uniform53(r0, r1)
    u2 = uniform53(r2, r3)
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * math.pi * u2
    return rad * np.cos(ang), rad * np.sin(ang)


def philox_uniform_int(index, tag, seed, lo, hi):
    """Deterministic integer in [lo, hi] (inclusive) for a given index/tag."""
    r0, r1, _, _ = philox4x32_10(np.uint32(index), 0, 0, np.uint32(tag), seed)
    u = uniform53(r0, r1)
    return int(lo + np.floor(u * (hi - lo + 1)))


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Config:
    """One synthetic workload.

    bands: ((count, lo, hi), ...) energy groups; occupied groups come first.
    nb / ni: uniform band count / product-basis size, or None with
    nb_range / ni_range giving the inclusive range of a seeded per-k / per-q
    draw (mirrored so that Nb_k = Nb_-k and NI_q = NI_-q).
    ntau: number of tau intervals (ntau + 1 points).  mesh: 'uniform' | 'upm'.
    """
    name: str
    grid: tuple
    bands: tuple
    nb: int | None
    ni: int | None
    ntau: int
    mesh: str
    beta: float
    niw_f: int
    niw_b: int
    nb_range: tuple | None = None
    ni_range: tuple | None = None
    upm_m: int = 5
    omega: float = 1.0
    seed: int = 1602
    dispersion: float = 0.05

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)

    # -- derived ------------------------------------------------------------
    @property
    def nk(self) -> int:
        return int(np.prod(self.grid))

    @property
    def ntau_points(self) -> int:
        return self.ntau + 1

    @property
    def scale(self) -> float:
        """s = -1 / (Omega N_k), the prefactor of P and Sigma."""
        return -1.0 / (self.omega * self.nk)


C1 = Config(name="c1_g0w0_fp64", grid=(2, 2, 2),
            bands=((8, -1.0, -0.05), (8, 0.05, 2.0)), nb=16, ni=64,
            ntau=32, mesh="uniform", beta=100.0, niw_f=32, niw_b=32)

C2 = Config(name="c2_k64_nb64_ni400", grid=(4, 4, 4),
            bands=((32, -1.0, -0.05), (32, 0.05, 2.0)), nb=64, ni=400,
            ntau=80, mesh="upm", beta=200.0, niw_f=128, niw_b=128)

_C3_BANDS = ((24, -3.0, -1.5), (40, -1.0, -0.05), (64, 0.05, 3.0))

C3 = Config(name="c3_k216_nb128_ni800", grid=(6, 6, 6), bands=_C3_BANDS,
            nb=128, ni=800, ntau=120, mesh="upm", beta=200.0,
            niw_f=128, niw_b=128)

C4 = Config(name="c4_k216_uneven", grid=(6, 6, 6),
            bands=((24, -3.0, -1.5), (40, -1.0, -0.05), (96, 0.05, 3.0)),
            nb=None, ni=None, nb_range=(96, 160), ni_range=(500, 900),
            ntau=120, mesh="upm", beta=200.0, niw_f=128, niw_b=128)

C5 = Config(name="c5_k125_nb128_ni700_scgw", grid=(5, 5, 5), bands=_C3_BANDS,
            nb=128, ni=700, ntau=160, mesh="upm", beta=400.0,
            niw_f=128, niw_b=128)

CONFIGS = {"c1": C1, "c2": C2, "c3": C3, "c4": C4, "c5": C5}


# ---------------------------------------------------------------------------
# k-grid
# ---------------------------------------------------------------------------
def kgrid(cfg: Config) -> np.ndarray:
    """Fractional k-vectors [nk, 3], index k = (i1*N2 + i2)*N3 + i3."""
    n1, n2, n3 = cfg.grid
    i = np.array([(a, b, c) for a in range(n1) for b in range(n2) for c in range(n3)])
    return i / np.array(cfg.grid, dtype=np.float64)


def _kindex(cfg, i1, i2, i3):
    n1, n2, n3 = cfg.grid
    return ((i1 % n1) * n2 + (i2 % n2)) * n3 + (i3 % n3)


def _kint(cfg):
    n1, n2, n3 = cfg.grid
    return np.array([(a, b, c) for a in range(n1) for b in range(n2) for c in range(n3)])


def kmq_table(cfg: Config) -> np.ndarray:
    """kmq[q, k] = index of k - q (mod the grid).  int32 [nk, nk]."""
    ki = _kint(cfg)
    nk = cfg.nk
    out = np.empty((nk, nk), dtype=np.int32)
    for q in range(nk):
        d = ki - ki[q]
        out[q] = _kindex(cfg, d[:, 0], d[:, 1], d[:, 2])
    return out


def minus_table(cfg: Config) -> np.ndarray:
    """minus[k] = index of -k (mod the grid)."""
    ki = _kint(cfg)
    return _kindex(cfg, -ki[:, 0], -ki[:, 1], -ki[:, 2]).astype(np.int32)


# ---------------------------------------------------------------------------
# tau mesh
# ---------------------------------------------------------------------------
def upm_mesh(beta: float, nint: int, m: int = 5) -> np.ndarray:
    if nint % (2 * m):
        raise ValueError("UPM needs ntau divisible by 2m")
    ph = nint // (2 * m)
    nodes = [0.0] + [(beta / 2.0) * 2.0 ** (j - ph) for j in range(1, ph + 1)]
    half = []
    for j in range(ph):
        a, b = nodes[j], nodes[j + 1]
        for i in range(m):
            half.append(a + (b - a) * i / m)
    half.append(beta / 2.0)
    tail = [beta - t for t in reversed(half[:-1])]
    return np.array(half + tail, dtype=np.float64)


def tau_mesh(cfg: Config) -> np.ndarray:
    if cfg.mesh == "uniform":
        t = np.linspace(0.0, cfg.beta, cfg.ntau + 1)
        # exact mirror symmetry
        n = cfg.ntau
        for i in range(n // 2 + 1):
            t[n - i] = cfg.beta - t[i]
        t[0], t[-1] = 0.0, cfg.beta
        return t
    if cfg.mesh == "upm":
        return upm_mesh(cfg.beta, cfg.ntau, cfg.upm_m)
    raise ValueError(cfg.mesh)


# ---------------------------------------------------------------------------
# band counts, product-basis sizes, energies, Coulomb kernel
# ---------------------------------------------------------------------------
def band_counts(cfg: Config) -> np.ndarray:
    nk = cfg.nk
    if cfg.nb is not None:
        return np.full(nk, cfg.nb, dtype=np.int32)
    lo, hi = cfg.nb_range
    mk = minus_table(cfg)
    out = np.zeros(nk, dtype=np.int32)
    for k in range(nk):
        c = min(k, int(mk[k]))
        out[k] = philox_uniform_int(c, TAG_NB, cfg.seed, lo, hi)
    return out


def basis_sizes(cfg: Config) -> np.ndarray:
    nk = cfg.nk
    if cfg.ni is not None:
        return np.full(nk, cfg.ni, dtype=np.int32)
    lo, hi = cfg.ni_range
    mk = minus_table(cfg)
    out = np.zeros(nk, dtype=np.int32)
    for q in range(nk):
        c = min(q, int(mk[q]))
        out[q] = philox_uniform_int(c, TAG_NI, cfg.seed, lo, hi)
    return out


def band_levels(cfg: Config) -> np.ndarray:
    """eps_n before dispersion: concatenated inclusive linspaces."""
    return np.concatenate([np.linspace(lo, hi, cnt) for cnt, lo, hi in cfg.bands])


def band_energies(cfg: Config) -> np.ndarray:
    """eps[k, n] (f64, [nk, nbmax]); entries n >= Nb_k are 0 and unused."""
    nb = band_counts(cfg)
    lev = band_levels(cfg)
    if nb.max() > lev.size:
        raise ValueError("band groups shorter than the band count")
    kv = kgrid(cfg)
    disp = cfg.dispersion * np.cos(2.0 * np.pi * kv).sum(axis=1)
    out = np.zeros((cfg.nk, int(nb.max())), dtype=np.float64)
    for k in range(cfg.nk):
        out[k, :nb[k]] = lev[:nb[k]] + disp[k]
    return out


def coulomb_v(cfg: Config) -> list:
    """v[q] = 4 pi / (0.1 + 0.09 I), I = 0..NI_q-1 (list of f64 arrays)."""
    ni = basis_sizes(cfg)
    return [4.0 * np.pi / (0.1 + 0.09 * np.arange(n, dtype=np.float64)) for n in ni]


def occupations0(eps: np.ndarray, nb: np.ndarray, beta: float, mu: float = 0.0):
    """Fermi occupations of the model levels at mu (input recipe for N_target)."""
    x = beta * (eps - mu)
    f = np.where(x >= 0, np.exp(-np.abs(x)) / (1.0 + np.exp(-np.abs(x))),
                 1.0 / (1.0 + np.exp(-np.abs(x))))
    mask = np.arange(eps.shape[1])[None, :] < nb[:, None]
    return np.where(mask, f, 0.0)


# ---------------------------------------------------------------------------
# matrix elements M
# ---------------------------------------------------------------------------
def m_layout(cfg: Config):
    """Per-q packing of M: for each q, blocks over k of shape
    [NI_q][Nb_k][Nb_{k-q}] (complex, row-major).  Returns (offsets[q][k] in
    complex elements relative to the start of q's block, size[q])."""
    nb = band_counts(cfg)
    ni = basis_sizes(cfg)
    kmq = kmq_table(cfg)
    nk = cfg.nk
    off = np.zeros((nk, nk + 1), dtype=np.int64)
    for q in range(nk):
        for k in range(nk):
            off[q, k + 1] = off[q, k] + int(ni[q]) * int(nb[k]) * int(nb[kmq[q, k]])
    return off[:, :-1].copy(), off[:, -1].copy()


class MGenerator:
    """Draws M blocks for a configuration (see the module docstring)."""

    def __init__(self, cfg: Config, seed: int | None = None, symmetric: bool = True):
        self.cfg = cfg
        self.seed = cfg.seed if seed is None else seed
        self.symmetric = symmetric
        self.nb = band_counts(cfg)
        self.ni = basis_sizes(cfg)
        self.kmq = kmq_table(cfg)
        self.minus = minus_table(cfg)
        self.nbmax = int(self.nb.max())
        # sub[a, b] = index of k_a - k_b
        self.sub = self.kmq.T.copy()

    def _lin(self, q, k, n, m):
        nk = self.cfg.nk
        nbm = np.uint64(self.nbmax)
        return ((np.uint64(q) * np.uint64(nk) + np.asarray(k, dtype=np.uint64)) * nbm
                + np.asarray(n, dtype=np.uint64)) * nbm + np.asarray(m, dtype=np.uint64)

    def block(self, q: int, k: int, dtype=np.complex128, rows=None) -> np.ndarray:
        """M^I_nm(k, q) as an array [NI_q, Nb_k, Nb_{k-q}] (or only the I in `rows`)."""
        nI = int(self.ni[q])
        nn = int(self.nb[k])
        kq = int(self.kmq[q, k])
        nm_ = int(self.nb[kq])
        n = np.arange(nn, dtype=np.uint64)[:, None]
        m = np.arange(nm_, dtype=np.uint64)[None, :]
        n, m = np.broadcast_arrays(n, m)
        x_e = self._lin(q, k, n, m)
        if self.symmetric:
            mq = int(self.minus[q])
            qmk = int(self.sub[q, k])          # q - k
            mk = int(self.minus[k])            # -k
            x_a = self._lin(q, qmk, m, n)
            x_b = self._lin(mq, mk, n, m)
            x_ab = self._lin(mq, kq, m, n)     # (-q, k - q, m, n)
            canon = np.minimum(np.minimum(x_e, x_a), np.minimum(x_b, x_ab))
            conj = (canon != x_e) & (canon != x_a)
            real = (x_b == x_e) | (x_ab == x_e)
        else:
            canon = x_e
            conj = np.zeros(x_e.shape, dtype=bool)
            real = np.zeros(x_e.shape, dtype=bool)
        I = (np.arange(nI, dtype=np.uint32) if rows is None
             else np.asarray(rows, dtype=np.uint32))[:, None, None]
        c0 = (canon & _U32).astype(np.uint32)[None]
        c1 = (canon >> np.uint64(32)).astype(np.uint32)[None]
        r0, r1, r2, r3 = philox4x32_10(c0, c1, I, np.uint32(TAG_M), self.seed)
        z0, z1 = box_muller(r0, r1, r2, r3)
        var = 1.0 / (1.0 + I.astype(np.float64) / 16.0)
        sc = np.sqrt(var / 2.0)
        re = np.where(real[None], np.sqrt(var) * z0, sc * z0)
        im = np.where(real[None], 0.0, np.where(conj[None], -sc * z1, sc * z1))
        return (re + 1j * im).astype(dtype)

    def q_blocks(self, q: int, dtype=np.complex128):
        return [self.block(q, k, dtype) for k in range(self.cfg.nk)]

    def q_packed(self, q: int, dtype=np.complex128) -> np.ndarray:
        """Flat packed M for one q, in the library layout."""
        return np.concatenate([b.reshape(-1) for b in self.q_blocks(q, dtype)])


# ---------------------------------------------------------------------------
# cubic crystal symmetry (input generation for the irreducible-wedge reduction)
# ---------------------------------------------------------------------------
TAG_MC = 0x4D435542       # matrix elements M of the cubic-symmetric generator


def cubic_group() -> np.ndarray:
    """The 48 signed permutation matrices (the point group O_h of a simple cubic lattice), int [48, 3, 3],
    the identity first."""
    out = []
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        for sgn in range(8):
            R = np.zeros((3, 3), dtype=np.int64)
            for r in range(3):
                R[r, perm[r]] = -1 if (sgn >> r) & 1 else 1
            out.append(R)
    return np.array(out)


def basis_vectors(ni: int) -> np.ndarray:
    """The first ni reciprocal-lattice vectors G in Z^3, ordered by |G|^2 then lexicographically
    (int [ni, 3]).  ni must close a shell, so that the set is mapped onto itself by O_h."""
    R = 1
    while (2 * R + 1) ** 3 < 4 * ni or R * R < np.cbrt(ni):
        R += 1
    g = np.array([(a, b, c) for a in range(-R, R + 1) for b in range(-R, R + 1) for c in range(-R, R + 1)])
    n2 = (g * g).sum(axis=1)
    order = np.lexsort((g[:, 2], g[:, 1], g[:, 0], n2))
    g, n2 = g[order], n2[order]
    if ni < g.shape[0] and n2[ni] == n2[ni - 1]:
        raise ValueError(f"NI = {ni} does not close a shell of reciprocal-lattice vectors")
    return g[:ni]


def rotation_k_maps(cfg: Config, group: np.ndarray | None = None) -> np.ndarray:
    """rot_k[r, k] = index of R_r k on the n x n x n grid (int32 [nrot, nk])."""
    group = cubic_group() if group is None else group
    n = cfg.grid[0]
    if not (cfg.grid[1] == n and cfg.grid[2] == n):
        raise ValueError("the cubic group acts on an n x n x n grid")
    ki = _kint(cfg)
    out = np.empty((group.shape[0], cfg.nk), dtype=np.int32)
    for r, R in enumerate(group):
        rk = ki @ R.T
        out[r] = _kindex(cfg, rk[:, 0], rk[:, 1], rk[:, 2])
    return out


def cubic_v(ni: int) -> np.ndarray:
    """v_I = 4 pi / (0.1 + 0.5 |G_I|^2): a function of |G| only, as the Coulomb kernel is."""
    g = basis_vectors(ni)
    return 4.0 * np.pi / (0.1 + 0.5 * (g * g).sum(axis=1).astype(np.float64))


class CubicGenerator:
    """M for an n x n x n grid with the symmetry of a symmorphic cubic crystal: the product basis is the
    set of the first NI vectors G (closed shells) and

        M^I'_nm(R k, R q) = M^I_nm(k, q)  with  G_I' = R G_I,  for all 48 R in O_h,

    the relation of the paper's symmetry subsection without fractional translations.  One complex
    Gaussian (E|M|^2 = 1 / (1 + |G|^2 / 4)) is drawn per orbit of (k, q, G) and band pair (n, m), keyed by
    the orbit's smallest index (q' nk + k') NI + I'.  Band counts and NI are the same at every k and q;
    the energies of the model bands are invariant under O_h."""

    def __init__(self, cfg: Config, seed: int | None = None):
        if cfg.nb is None or cfg.ni is None:
            raise ValueError("the cubic generator needs uniform band counts and basis size")
        self.cfg = cfg
        self.seed = cfg.seed if seed is None else seed
        self.group = cubic_group()
        self.rot_k = rotation_k_maps(cfg, self.group)
        self.g = basis_vectors(cfg.ni)
        self.nb = band_counts(cfg)
        self.ni = basis_sizes(cfg)
        self.kmq = kmq_table(cfg)
        R = int(np.abs(self.g).max())
        self._R = R
        look = -np.ones((2 * R + 1,) * 3, dtype=np.int64)
        look[self.g[:, 0] + R, self.g[:, 1] + R, self.g[:, 2] + R] = np.arange(cfg.ni)
        self._look = look
        # rot_g[r, I] = index of R_r G_I
        rg = np.einsum("rij,gj->rgi", self.group, self.g) + R
        self.rot_g = look[rg[..., 0], rg[..., 1], rg[..., 2]]
        assert (self.rot_g >= 0).all()

    def keys(self, q: int) -> np.ndarray:
        """Orbit key of every (k, I) of q: uint64 [nk, NI]."""
        nk, ni = self.cfg.nk, self.cfg.ni
        qq = self.rot_k[:, q].astype(np.uint64)[:, None, None]            # [r, 1, 1]
        kk = self.rot_k.astype(np.uint64)[:, :, None]                       # [r, k, 1]
        ii = self.rot_g.astype(np.uint64)[:, None, :]                       # [r, 1, I]
        key = (qq * np.uint64(nk) + kk) * np.uint64(ni) + ii
        return key.min(axis=0)

    def block(self, q: int, k: int, dtype=np.complex128, keys=None) -> np.ndarray:
        nb = self.cfg.nb
        key = (self.keys(q) if keys is None else keys)[k][:, None, None]     # [I, 1, 1]
        nm = (np.arange(nb, dtype=np.uint32)[:, None] * np.uint32(nb) + np.arange(nb, dtype=np.uint32)[None, :])
        c0 = (key & _U32).astype(np.uint32)
        c1 = (key >> np.uint64(32)).astype(np.uint32)
        r0, r1, r2, r3 = philox4x32_10(c0, c1, nm[None], np.uint32(TAG_MC), self.seed)
        z0, z1 = box_muller(r0, r1, r2, r3)
        g2 = (self.g * self.g).sum(axis=1).astype(np.float64)[:, None, None]
        sc = np.sqrt(1.0 / (1.0 + g2 / 4.0) / 2.0)
        return (sc * z0 + 1j * sc * z1).astype(dtype)

    def q_blocks(self, q: int, dtype=np.complex128):
        keys = self.keys(q)
        return [self.block(q, k, dtype, keys) for k in range(self.cfg.nk)]

    def q_packed(self, q: int, dtype=np.complex128) -> np.ndarray:
        return np.concatenate([b.reshape(-1) for b in self.q_blocks(q, dtype)])


def make_cubic_problem(cfg: Config) -> "Problem":
    """A Problem whose Coulomb kernel is the cubic generator's v (a function of |G|)."""
    prob = make_problem(cfg)
    prob.v = [cubic_v(int(n)) for n in prob.ni]
    return prob


@dataclass
class Problem:
    """Everything a run needs, derived from a Config."""
    cfg: Config
    nb: np.ndarray
    ni: np.ndarray
    kmq: np.ndarray
    tau: np.ndarray
    eps: np.ndarray
    v: list
    n_target: float
    m_offsets: np.ndarray = field(repr=False)
    m_sizes: np.ndarray = field(repr=False)


def make_problem(cfg: Config) -> Problem:
    nb = band_counts(cfg)
    ni = basis_sizes(cfg)
    eps = band_energies(cfg)
    off, sz = m_layout(cfg)
    f = occupations0(eps, nb, cfg.beta, 0.0)
    return Problem(cfg=cfg, nb=nb, ni=ni, kmq=kmq_table(cfg), tau=tau_mesh(cfg),
                   eps=eps, v=coulomb_v(cfg), n_target=float(f.sum()),
                   m_offsets=off, m_sizes=sz)


def tiny(name="tiny", grid=(2, 1, 1), nocc=2, nemp=2, ni=5, ntau=12, beta=20.0,
         niw=16, mesh="uniform", **kw) -> Config:
    """Small configurations for tests."""
    return Config(name=name, grid=grid,
                  bands=((nocc, -1.0, -0.1), (nemp, 0.1, 1.5)) if nemp else ((nocc, -1.0, -0.1),),
                  nb=nocc + nemp, ni=ni, ntau=ntau, mesh=mesh, beta=beta,
                  niw_f=niw, niw_b=niw, **kw)
