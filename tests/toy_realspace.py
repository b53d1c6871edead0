"""Real-space brute-force toy used to pin the oracle's P, W~, Sigma^c and Sigma^x.

A 1D chain (lattice constant 1) with N_k = 2 k-points (k = 0, pi) and Nr = 4
grid points per cell: the 8-point supercell has an 8-dimensional Hilbert space
spanned by the 2 x 4 Bloch states, and the 8 plane waves e^{i p x}, p = 2 pi
(q + g), g = 0..3, form a complete product basis.  Everything is computed in
real space from the paper's real-space definitions and then projected:

* G(r, r', tau) = sum_kn psi_nk(r) G_n(k, tau) psi*_nk(r')        (Bloch expansion of G)
* P(r, r', tau) = G(r, r', tau) G(r', r, -tau), G(-tau) = -G(beta - tau)   (eq. prr)
* W~ = (1 - v P)^-1 v P v on the Matsubara axis, products over r        (eq. scrv)
* Sigma^c(r, r', tau) = -G(r, r', tau) W~(r, r', tau)                    (eq. gw1)
* Sigma^x(r, r') = -rho(r, r') v(r, r'), rho = G(tau -> 0-)              (Sigma^x = -G v delta)

With M = sqrt(Ns) sum_r psi*_{m,k-q} e^{-i p x} psi_{nk}, Omega = Nr and
v_lib = v_p / Ns the product-basis formulas of the oracle must reproduce the
projections exactly; this pins the sign, the conjugate placement, which G
carries tau and which beta - tau, and the 1/(Omega N_k) normalisation.
"""
import numpy as np

NK = 2
NR = 4
NS = NK * NR


class Toy:
    def __init__(self, seed=7, nb=4, beta=10.0, ntau=21):
        rng = np.random.default_rng(seed)
        self.beta = beta
        self.tau = np.linspace(0.0, beta, ntau)
        self.tau[-1] = beta
        self.x = np.arange(NS) / NR                       # positions, supercell length 2
        self.kfrac = np.array([0.0, 0.5])
        self.nb = nb
        # band energies (2 occupied, 2 empty) and random unitary Bloch parts
        self.eps = np.array([[-0.9, -0.3, 0.4, 1.1], [-0.7, -0.2, 0.6, 1.3]])[:, :nb]
        self.psi = np.zeros((NK, nb, NS), dtype=np.complex128)
        for k in range(NK):
            Z = rng.normal(size=(NR, NR)) + 1j * rng.normal(size=(NR, NR))
            U, _ = np.linalg.qr(Z)
            for n in range(nb):
                u = np.tile(U[:, n], NK) / np.sqrt(NK)
                self.psi[k, n] = np.exp(2j * np.pi * self.kfrac[k] * self.x) * u
        # product basis p_{q, I} = 2 pi (q + g_I)
        self.g = np.arange(NR)
        self.p = 2 * np.pi * (self.kfrac[:, None] + self.g[None, :])      # [q, I]
        self.vp = 1.0 / (0.3 + (self.p / (2 * np.pi)) ** 2)                 # any positive
        self.v_lib = self.vp / NS
        self.kmq = np.array([[(k - q) % NK for k in range(NK)] for q in range(NK)])
        self.s = -1.0 / (NR * NK)                        # -1/(Omega N_k), Omega = Nr
        # matrix elements M^I_nm(k, q)
        self.M = [[None] * NK for _ in range(NK)]
        for q in range(NK):
            for k in range(NK):
                kq = self.kmq[q, k]
                ph = np.exp(-1j * np.outer(self.p[q], self.x))             # [I, r]
                # sum_r conj(psi_m,k-q(r)) e^{-ipx} psi_nk(r)
                self.M[q][k] = np.sqrt(NS) * np.einsum("mr,ir,nr->inm",
                                                        self.psi[kq].conj(), ph, self.psi[k])
        # plane waves b_p(r) per q: [I, r]
        self.pw = [np.exp(1j * np.outer(self.p[q], self.x)) for q in range(NK)]

    # -- real-space objects ---------------------------------------------------
    def G_bands(self, G0fun):
        return np.stack([G0fun(self.eps[k]) for k in range(NK)])        # [k, n, tau]

    def G_real(self, Gb):
        # [tau, r, r']
        return np.einsum("knr,knt,kns->trs", self.psi, Gb, self.psi.conj())

    def P_real(self, Gb):
        Gr = self.G_real(Gb)
        N = Gr.shape[0]
        out = np.empty_like(Gr)
        for i in range(N):
            # G(r, r', tau) * G(r', r, -tau) with G(-tau) = -G(beta - tau)
            out[i] = Gr[i] * (-Gr[N - 1 - i].T)
        return out

    def project_pair(self, A, q):
        """sum_rr' e^{-i p_I x_r} A(r, r') e^{i p_J x_r'} for one q."""
        ph = self.pw[q]
        return np.einsum("ir,...rs,js->...ij", ph.conj(), A, ph)

    def v_real(self):
        out = np.zeros((NS, NS), dtype=np.complex128)
        for q in range(NK):
            ph = self.pw[q]
            out += np.einsum("ir,i,is->rs", ph, self.vp[q], ph.conj()) / NS
        return out

    def W_real_from_lib(self, Wlib):
        """Real-space W~(r, r') from per-q product-basis blocks W~_lib[q] ([..., I, J])."""
        out = 0
        for q in range(NK):
            ph = self.pw[q]
            out = out + np.einsum("ir,...ij,js->...rs", ph, Wlib[q], ph.conj())
        return out

    def project_bands(self, A, k):
        """sum_rr' psi*_nk(r) A(r, r') psi_n'k(r')."""
        return np.einsum("nr,...rs,ps->...np", self.psi[k].conj(), A, self.psi[k])
