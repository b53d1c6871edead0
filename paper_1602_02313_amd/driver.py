"""Device-resident driver of the Matsubara-time GW loop (one GPU).

Owns the torch buffers and sequences the C-ABI calls; every step of the path
runs in libmatsgw's kernels.  Loop structure of the paper's "Scheme for scGW"
subsection: G0W0 is the first pass, GW0 keeps W~ from the first iteration and
scGW updates everything.
"""
from __future__ import annotations

import contextlib
from collections import defaultdict

import numpy as np

from . import _lib as L


class HostM:
    """M from host arrays: q -> flat complex numpy array in the library layout."""

    def __init__(self, per_q, dtype):
        self.per_q = per_q
        self.dtype = dtype
        self._cache = {}

    def __call__(self, run, q0, nq):
        import torch
        key = (q0, nq)
        if key not in self._cache:
            flat = np.concatenate([np.asarray(self.per_q(q)).reshape(-1) for q in range(q0, q0 + nq)])
            ct = torch.complex128 if self.dtype == L.C128 else torch.complex64
            self._cache = {key: torch.from_numpy(flat).to(ct).to(run.device)}
        return self._cache[key]


class ResidentM:
    """All q blocks resident in one device tensor (complex, library layout)."""

    def __init__(self, tensor, mpre):
        self.t = tensor
        self.mpre = mpre

    def __call__(self, run, q0, nq):
        return self.t[self.mpre[q0]:self.mpre[q0 + nq]]


class SynthM:
    """M generated on the device per q batch by msgw_synth_M (Philox4x32-10)."""

    def __init__(self, seed, symmetric=True):
        self.seed = seed
        self.symmetric = symmetric
        self.buf = None

    def reserve(self, run):
        """Allocate the buffer for the largest q batch of `run` (before a graph capture)."""
        import torch
        size = max(int(run.mpre[q0 + nq] - run.mpre[q0]) for q0, nq in run._batches())
        ct = torch.complex128 if run.m_dtype == L.C128 else torch.complex64
        if self.buf is None or self.buf.numel() < size or self.buf.dtype != ct:
            self.buf = torch.empty(size, dtype=ct, device=run.device)

    def __call__(self, run, q0, nq):
        import torch
        size = int(run.mpre[q0 + nq] - run.mpre[q0])
        ct = torch.complex128 if run.m_dtype == L.C128 else torch.complex64
        if self.buf is None or self.buf.numel() < size or self.buf.dtype != ct:
            self.buf = torch.empty(size, dtype=ct, device=run.device)
        out = self.buf[:size]
        run.ctx.synth_M(self.seed, q0, nq, self.symmetric, run.m_dtype, out, stream=run.stream)
        return out


class SynthCubicM(SynthM):
    """M with the symmetry of a cubic crystal, generated on the device by msgw_synth_M_cubic."""

    def __init__(self, seed):
        super().__init__(seed, True)

    def __call__(self, run, q0, nq):
        import torch
        size = int(run.mpre[q0 + nq] - run.mpre[q0])
        ct = torch.complex128 if run.m_dtype == L.C128 else torch.complex64
        if self.buf is None or self.buf.numel() < size or self.buf.dtype != ct:
            self.buf = torch.empty(size, dtype=ct, device=run.device)
        out = self.buf[:size]
        run.ctx.synth_M_cubic(self.seed, q0, nq, run.m_dtype, out, stream=run.stream)
        return out


class EventTimer:
    """HIP events recorded around each library call on the launch stream.

    With ctx given, the polarization and self-energy calls also get a pair of events that the library
    records around their contraction kernels alone (msgw_set_kernel_events), on the same stream."""

    KERNEL_OPS = {"polarization": L.OP_POLARIZATION, "self_energy": L.OP_SELF_ENERGY}

    def __init__(self, stream=None, ctx=None):
        import torch
        self.torch = torch
        self.stream = stream
        self.ctx = ctx
        self.events = defaultdict(list)
        self.kernel_events = defaultdict(list)

    @contextlib.contextmanager
    def __call__(self, name):
        T = self.torch
        st = self.stream if self.stream is not None else T.cuda.current_stream()
        a, b = T.cuda.Event(enable_timing=True), T.cuda.Event(enable_timing=True)
        op = self.KERNEL_OPS.get(name) if self.ctx is not None else None
        if op is not None:
            ka, kb = T.cuda.Event(enable_timing=True), T.cuda.Event(enable_timing=True)
            ka.record(st)  # creates the events; the library records them again around its kernels
            kb.record(st)
            self.ctx.set_kernel_events(op, ka, kb)
        a.record(st)
        try:
            yield
        finally:
            b.record(st)
            if op is not None:
                self.ctx.set_kernel_events(op)
        self.events[name].append((a, b))
        if op is not None:
            self.kernel_events[name].append((ka, kb))

    def reset(self):
        self.events.clear()
        self.kernel_events.clear()

    def summary(self):
        """name -> list of durations in ms (synchronises)."""
        self.torch.cuda.synchronize()
        return {k: [a.elapsed_time(b) for a, b in v] for k, v in self.events.items()}

    def kernel_summary(self):
        """name -> list of durations in ms of the contraction kernels alone (synchronises)."""
        self.torch.cuda.synchronize()
        return {k: [a.elapsed_time(b) for a, b in v] for k, v in self.kernel_events.items()}


class GWRun:
    """State of one run: problem tables, workspace, G, Sigma and per-q-batch buffers."""

    def __init__(self, nk, kmq, nb, ni, tau, beta, niw_f, niw_b, scale, eps, v, n_target,
                 precision=L.FP64, sigma_mode=L.SIGMA_DIAG, q_batch=1, device=0, stream=None,
                 tau_mirror=False):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = stream
        self.nk = int(nk)
        self.nb = np.asarray(nb, dtype=np.int32)
        self.ni = np.asarray(ni, dtype=np.int32)
        self.kmq = np.asarray(kmq, dtype=np.int32).reshape(self.nk, self.nk)
        self.tau = np.asarray(tau, dtype=np.float64)
        self.ntau = self.tau.size
        self.beta = float(beta)
        self.niw_f, self.niw_b = int(niw_f), int(niw_b)
        self.nbmax = int(self.nb.max())
        self.precision = precision
        self.sigma_mode = sigma_mode
        self.m_dtype = L.C128 if precision == L.FP64 else L.C64
        self.n_target = float(n_target)
        self.q_batch = int(q_batch)
        self.ctx = L.Context(device)
        self.ctx.set_problem(self.nk, self.kmq, self.nb, self.ni, self.tau, self.beta,
                             self.niw_f, self.niw_b, scale, sigma_mode)
        ws_bytes = self.ctx.workspace_size(self.q_batch)
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)
        self.ctx.set_workspace(self.ws)
        if tau_mirror:  # the caller asserts P(tau) = P(beta - tau) for its inputs
            self.ctx.set_tau_mirror(True)
        # prefixes of the packed per-q arrays
        nk = self.nk
        self.mpre = np.zeros(nk + 1, dtype=np.int64)
        for q in range(nk):
            self.mpre[q + 1] = self.mpre[q] + self.ctx.m_layout(q, nk)[1]
        self.ppre = np.concatenate([[0], np.cumsum(self.ntau * self.ni.astype(np.int64) ** 2)])
        self.wpre = np.concatenate([[0], np.cumsum(self.niw_b * self.ni.astype(np.int64) ** 2)])
        self.vpre = np.concatenate([[0], np.cumsum(self.ni.astype(np.int64))])
        f64, c128 = torch.float64, torch.complex128
        dev = self.device
        self.eps = torch.from_numpy(np.ascontiguousarray(eps, dtype=np.float64)).to(dev)
        self.v = torch.from_numpy(np.concatenate([np.asarray(x, dtype=np.float64) for x in v])).to(dev)
        self.G_tau = torch.zeros((nk, self.nbmax, self.ntau), dtype=f64, device=dev)
        if sigma_mode == L.SIGMA_FULL:
            self.sig_tau = torch.zeros((nk, self.nbmax, self.nbmax, self.ntau), dtype=c128, device=dev)
            self.sig_x = torch.zeros((nk, self.nbmax, self.nbmax), dtype=c128, device=dev)
        else:
            self.sig_tau = torch.zeros((nk, self.nbmax, self.ntau), dtype=f64, device=dev)
            self.sig_x = torch.zeros((nk, self.nbmax), dtype=f64, device=dev)
        self.sig_iw = torch.zeros((nk, self.nbmax, self.niw_f), dtype=c128, device=dev)
        self.G_iw = torch.zeros((nk, self.nbmax, self.niw_f), dtype=c128, device=dev)
        self.mu = torch.zeros(1, dtype=f64, device=dev)
        self.N = torch.zeros(1, dtype=f64, device=dev)
        self.gap_d = torch.zeros(1, dtype=f64, device=dev)
        self.flags = torch.zeros(1, dtype=torch.int32, device=dev)
        self.screen_flags = torch.zeros(1, dtype=torch.int32, device=dev)  # MSGW_FLAG_SINGULAR of a pass
        # per q batch
        maxp = max(int(self.ppre[q + self.q_batch] - self.ppre[q])
                   for q in range(0, nk - self.q_batch + 1)) if nk >= self.q_batch else int(self.ppre[-1])
        maxw = max(int(self.wpre[q + self.q_batch] - self.wpre[q])
                   for q in range(0, nk - self.q_batch + 1)) if nk >= self.q_batch else int(self.wpre[-1])
        self.P_tau = torch.empty(maxp, dtype=c128, device=dev)
        self.Wt_tau = torch.empty(maxp, dtype=c128, device=dev)
        self.P_iw = torch.empty(maxw, dtype=c128, device=dev)
        self.Wt_iw = torch.empty(maxw, dtype=c128, device=dev)
        self.R_iw = torch.empty(maxw, dtype=c128, device=dev)
        self.info = torch.zeros(self.q_batch * self.niw_b, dtype=torch.int32, device=dev)
        self.W_frozen = None
        self.timer = None
        self.ibz = None  # irreducible q (set_symmetry): the passes run over these and their stars

    def set_symmetry(self, rot_k):
        """Use the point group given by its action on the k grid (rot_k[r][k] = index of R_r k): the
        self-energy passes then compute P, W~ and the contractions for the irreducible q only and add
        each one's contributions over its star (msgw_sigma_star).  DIAG mode."""
        import torch
        self.ctx.set_symmetry(rot_k)
        self.ibz, self.star_size = self.ctx.ibz()
        self.C_tau = torch.zeros_like(self.sig_tau)
        self.C_x = torch.zeros_like(self.sig_x)

    def _t(self, name):
        return self.timer(name) if self.timer is not None else contextlib.nullcontext()

    # -- steps ---------------------------------------------------------------------------------
    def green0(self, mu=0.0):
        with self._t("green0"):
            self.ctx.green0(self.eps, mu, self.G_tau, stream=self.stream)

    def _batches(self):
        q = 0
        while q < self.nk:
            nq = min(self.q_batch, self.nk - q)
            yield q, nq
            q += nq

    def q_block(self, M_source, q0, nq, keep=None):
        """P -> P(i nu) -> W~(i nu) -> W~(tau) -> Sigma^c, Sigma^x for q0..q0+nq-1."""
        ctx, st = self.ctx, self.stream
        M = M_source(self, q0, nq)
        if self.W_frozen is None or q0 not in self.W_frozen:
            with self._t("polarization"):
                ctx.polarization(q0, nq, M, self.m_dtype, self.G_tau, self.precision, self.P_tau,
                                 stream=st)
            with self._t("tau_to_iw_P"):
                if len(set(int(x) for x in self.ni[q0:q0 + nq])) == 1:
                    # equal NI: the q blocks form one [nq][ntau][NI^2] batch
                    n = int(self.ni[q0])
                    ctx.tau_to_iw(L.BOSON, nq, n * n, self.P_tau, 1, None, self.P_iw, stream=st)
                else:
                    for q in range(q0, q0 + nq):
                        n = int(self.ni[q])
                        p0 = int(self.ppre[q] - self.ppre[q0])
                        w0 = int(self.wpre[q] - self.wpre[q0])
                        ctx.tau_to_iw(L.BOSON, 1, n * n, self.P_tau[p0:], 1, None, self.P_iw[w0:],
                                      stream=st)
            with self._t("screen"):
                ctx.screen(q0, nq, self.P_iw, self.v[self.vpre[q0]:], self.Wt_iw, self.R_iw,
                           self.info, self.screen_flags, stream=st)
            with self._t("screened_tau"):
                ctx.screened_tau(q0, nq, self.R_iw, self.P_tau, self.v[self.vpre[q0]:],
                                 self.Wt_tau, stream=st)
            Wt = self.Wt_tau
            if keep is not None:
                keep[q0] = self.Wt_tau[:int(self.ppre[q0 + nq] - self.ppre[q0])].clone()
        else:
            Wt = self.W_frozen[q0]
        with self._t("self_energy"):
            ctx.self_energy(q0, nq, M, self.m_dtype, self.G_tau, Wt, self.precision, self.sig_tau,
                            stream=st)
        with self._t("sigma_x"):
            ctx.sigma_x(q0, nq, M, self.m_dtype, self.G_tau, self.v[self.vpre[q0]:], self.sig_x,
                        stream=st)

    def begin_pass(self):
        """Zero the accumulated Sigma^c(tau), Sigma^x (and the screens' flags) before the q blocks."""
        self.sig_tau.zero_()
        self.sig_x.zero_()
        if self.W_frozen is None:  # with W~ frozen (GW0) the flags of its pass stay
            self.screen_flags.zero_()

    def sigma_to_iw(self):
        """Sigma^c(tau) -> Sigma^c(i w) after the last q block of a pass."""
        if self.sigma_mode == L.SIGMA_DIAG:
            with self._t("tau_to_iw_sigma"):
                self.ctx.tau_to_iw(L.FERMION, self.nk * self.nbmax, 1, self.sig_tau, 0, None,
                                   self.sig_iw, stream=self.stream)

    def q_block_star(self, M_source, q, keep=None):
        """An irreducible q: P, W~ and its contributions to every k, added over its star."""
        self.C_tau.zero_()
        self.C_x.zero_()
        sig, sx = self.sig_tau, self.sig_x
        self.sig_tau, self.sig_x = self.C_tau, self.C_x
        try:
            self.q_block(M_source, q, 1, keep=keep)
        finally:
            self.sig_tau, self.sig_x = sig, sx
        with self._t("sigma_star"):
            self.ctx.sigma_star(q, self.C_tau, self.C_x, self.sig_tau, self.sig_x, stream=self.stream)

    def sigma_pass(self, M_source, keep_W=False):
        """Sigma^c(tau), Sigma^x and Sigma^c(i w) from the current G (all q, or the irreducible q and
        their stars once set_symmetry was called)."""
        self.begin_pass()
        keep = {} if keep_W else None
        if self.ibz is not None:
            for q in self.ibz:
                self.q_block_star(M_source, q, keep=keep)
        else:
            for q0, nq in self._batches():
                self.q_block(M_source, q0, nq, keep=keep)
        if keep_W:
            self.W_frozen = keep
        self.sigma_to_iw()

    def dyson(self, search=True):
        with self._t("dyson"):
            self._dyson(search)

    def _dyson(self, search):
        self.ctx.dyson(self.eps, self.sig_x, self.sig_iw, self.n_target,
                       L.MU_SEARCH if search else L.MU_FIXED, self.mu, self.G_iw, self.G_tau,
                       self.N, self.flags, stream=self.stream)

    def gap(self):
        with self._t("gap"):
            self._gap()

    def _gap(self):
        self.ctx.gap(self.eps, self.sig_x, self.sig_iw, self.mu, int(round(self.n_target)),
                     self.gap_d, stream=self.stream)

    def continue_pade(self, n_pade=16, eta=0.0, omega=None):
        """Pade continuation of the current Sigma^c(i w) (after the path): quasiparticle energies,
        their gap, and A(w) on the real grid omega (energies from mu) when given.

        Returns (E_qp [nk, nbmax], A [nk, nbmax, n_omega] or None, gap, flags)."""
        import torch
        dev, f64 = self.device, torch.float64
        E = torch.empty((self.nk, self.nbmax), dtype=f64, device=dev)
        om = None if omega is None else torch.as_tensor(omega, dtype=f64).to(dev).contiguous()
        A = None if om is None else torch.empty((self.nk, self.nbmax, om.numel()), dtype=f64, device=dev)
        flags = torch.zeros(1, dtype=torch.int32, device=dev)
        gap = torch.zeros(1, dtype=f64, device=dev)
        self.ctx.continue_pade(n_pade, eta, self.eps, self.sig_x, self.sig_iw, self.mu, om, A, E, flags,
                               stream=self.stream)
        self.ctx.gap_of(E, int(round(self.n_target)), gap, stream=self.stream)
        return E, A, gap, flags

    def continue_cpe(self, n_real=61, w_min=-3.0, w_max=3.0, ridge=1e-10, eta=0.02, omega=None):
        """CPE continuation of the current Sigma^c(i w): quasiparticle energies, their gap, the fitted
        coefficients, and A(w) on omega when given.  Returns (E_qp, A or None, gap, coef, flags)."""
        import torch
        dev, f64 = self.device, torch.float64
        E = torch.empty((self.nk, self.nbmax), dtype=f64, device=dev)
        coef = torch.empty((self.nk, self.nbmax, n_real - 2), dtype=f64, device=dev)
        om = None if omega is None else torch.as_tensor(omega, dtype=f64).to(dev).contiguous()
        A = None if om is None else torch.empty((self.nk, self.nbmax, om.numel()), dtype=f64, device=dev)
        flags = torch.zeros(1, dtype=torch.int32, device=dev)
        gap = torch.zeros(1, dtype=f64, device=dev)
        self.ctx.continue_cpe(n_real, w_min, w_max, ridge, eta, self.eps, self.sig_x, self.sig_iw, self.mu, om, A,
                              E, coef, flags, stream=self.stream)
        self.ctx.gap_of(E, int(round(self.n_target)), gap, stream=self.stream)
        return E, A, gap, coef, flags

    def _record(self):
        """Host copies of mu, N, the gap proxy and the status bits (MSGW_FLAG_*) of the Dyson step
        and of the screens of the last pass."""
        return dict(mu=float(self.mu.item()), N=float(self.N.item()),
                    gap=float(self.gap_d.item()),
                    flags=int(self.flags.item()) | int(self.screen_flags.item()))

    def iteration(self, M_source, search=True):
        """One self-consistent iteration: Sigma from the current G, Dyson with the mu search, gap."""
        self.sigma_pass(M_source)
        self.dyson(search)
        self.gap()

    def capture_iteration(self, M_source, search=True):
        """The scGW iteration recorded once as a HIP graph (torch.cuda.CUDAGraph).

        Every step is a kernel launch or a device fill on the capture stream, so replaying the
        graph repeats the iteration from the current device state (G, mu) without host work.
        The M source must live on the device: ResidentM, or SynthM (its buffer is reserved here).
        """
        import torch
        if isinstance(M_source, HostM):
            raise ValueError("graph capture needs a device-resident M source (ResidentM or SynthM)")
        if self.stream is not None:
            raise ValueError("graph capture runs on torch's capture stream; construct GWRun with stream=None")
        if isinstance(M_source, SynthM):
            M_source.reserve(self)
        timer, self.timer = self.timer, None
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.iteration(M_source, search)
        torch.cuda.synchronize()
        self.timer = timer
        return g

    def run(self, M_source, mode="g0w0", niter=1, graph=False):
        """Returns a list of per-iteration dicts (host copies of mu, N, gap, flags).

        graph=True (scGW only): the iteration is captured once and replayed niter times.
        """
        self.green0(0.0)
        self.mu.zero_()
        self.W_frozen = None
        hist = []
        if graph and mode == "scgw":
            g = self.capture_iteration(M_source)
            for _ in range(niter):
                g.replay()
                hist.append(self._record())
            return hist
        for it in range(1 if mode == "g0w0" else niter):
            self.sigma_pass(M_source, keep_W=(mode == "gw0" and it == 0))
            if mode != "g0w0":
                self.dyson(True)
            self.gap()
            hist.append(self._record())
        return hist
