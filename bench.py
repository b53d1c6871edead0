#!/usr/bin/env python3
"""Benchmark of the Matsubara-time GW hot path on one MI355X.

The timed work is ONE self-consistent (scGW) iteration of the 5x5x5 k-grid, 128-band, NI = 700,
161-point power-mesh workload at beta = 400: for every q, M(q) is drawn on the device from the seed
(11.5 GB per q in complex64), then P(q,tau) -> P(q,i nu) -> W~(q,i nu) -> W~(q,tau) -> Sigma^c(k,tau)
and Sigma^x accumulate; after the last q, Sigma^c(k,i omega), the Dyson update with the
chemical-potential search and the gap proxy.  The K timed steps split that iteration: step s runs
the q in [s nk / K, (s + 1) nk / K) and the last step also runs the Dyson part, so K steps are
exactly one iteration and ms_per_step * K is the time of one iteration.  The warm-up steps run the
first W slices of an iteration that is then started over.

The metric is the P + Sigma effective TFLOP/s of the dense complex flop model (8 real flops per
complex multiply-add) over the whole iteration, and the seconds per iteration.  The roofline object
is the dominant contraction kernel's executed MFMA work (counted from the kernel's loop structure,
the Hermitian triangle and tile padding included) over its time, measured with HIP events that the
library records around its kernels, against MI355X's dense fp16/bf16 MFMA peak.

    python bench.py [--steps K] [--warmup W] [--config c5] [--precision f16x3|bf16x3|fp32|fp64]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# dense MFMA peaks of MI355X (TFLOP/s).  A split product costs three 16-bit products, so the split
# paths' FP32-equivalent peak is the 16-bit peak / 3.
PEAK_16 = 2516.6
PEAK = {"f16x3": PEAK_16 / 3.0, "bf16x3": PEAK_16 / 3.0, "fp32": 157.3, "fp64": 78.6}
MFMA_32X32X16 = 2 * 32 * 32 * 16   # flops of one v_mfma_f32_32x32x16_{f16,bf16}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------------------------
# work models (host logic; tested on the CPU)
# ---------------------------------------------------------------------------------------------
def flop_model(prob, qs=None, ks=None):
    """Dense complex flop counts (F_P, F_Sigma) of the q in qs (default all) over the k in ks."""
    cfg = prob.cfg
    ntau = prob.tau.size
    qs = range(cfg.nk) if qs is None else qs
    ks = range(cfg.nk) if ks is None else ks
    fp = fs = 0.0
    for q in qs:
        ni = int(prob.ni[q])
        for k in ks:
            nn, nm = int(prob.nb[k]), int(prob.nb[prob.kmq[q, k]])
            fp += 8.0 * ni * ni * nn * nm * ntau
            fs += 8.0 * ni * ni * nn * nm * ntau + 8.0 * ni * nn * nm * ntau
    return fp, fs


# the pair-space kernels: (WI, KS) of the polarization variants, by name
POLZ_SHAPES = {
    "pair-space 16x16 pairs K64 st4x8 3-buffer": (4, 64),
    "pair-space 16x16 pairs K64 3-buffer persistent LPT queue": (4, 64),
    "pair-space 16x16 pairs K64 st4x8": (4, 64),
    "pair-space 8x16 pairs 2 WG/CU st4x16 K64": (2, 64),
    "pair-space 8x16 pairs 2 WG/CU st4x16": (2, 32),
}
SIGZ_NAMES = ("pair-space 512 K x 8x8-pair blocks", "pair-space 512 K x 8x8-pair blocks persistent LPT queue")


def _tau_chunks(ntau):
    """Tile counts NTT of the 96-wide tau chunks and the tail chunk (32-wide MFMA tiles)."""
    nt = -(-ntau // 32)
    return [3] * (nt // 3) + ([nt % 3] if nt % 3 else [])


def executed_mfma_flops(prob, op, tile, q0, nq):
    """MFMA flops the pair-space kernel executes for one call over q0..q0+nq-1 (None for a tile
    form without a model).  Counted from the kernels' loops: the polarization runs, per work item
    (a block of 4 WI rows I x 16 columns J touching the upper triangle, and a tau chunk of NTT
    tiles), 2 WI waves x K_pad / 16 steps per k x 6 NTT MFMAs of 32x32x16; the self-energy runs,
    per (q, k, 512-row chunk of K, tau chunk), 8 waves x (upper-triangle 8x8-pair blocks) x 8 steps
    x 6 NTT MFMAs."""
    cfg = prob.cfg
    ntau = prob.tau.size
    chunks = _tau_chunks(ntau)
    n = 0
    for q in range(q0, q0 + nq):
        NI = int(prob.ni[q])
        Ks = [int(prob.nb[k]) * int(prob.nb[prob.kmq[q, k]]) for k in range(cfg.nk)]
        if op == 0:
            if tile not in POLZ_SHAPES:
                return None
            WI, _ = POLZ_SHAPES[tile]
            steps = sum(-(-K // 64) * 64 // 16 for K in Ks)
            items = 0
            for r in range(-(-NI // (4 * WI))):
                I0 = 4 * WI * r
                items += sum(1 for cj in range(-(-NI // 16)) if 16 * cj + 16 > I0)
            n += items * 2 * WI * steps * 6 * sum(chunks)
        else:
            if tile not in SIGZ_NAMES:
                return None
            n8 = -(-NI // 8)
            nblk = n8 * (n8 + 1) // 2
            kchunks = sum(-(-K // 512) for K in Ks)
            n += kchunks * 8 * nblk * 8 * 6 * sum(chunks)
    return float(n) * MFMA_32X32X16


def iteration_slices(nk, steps):
    """The q range [a, b) of each of the `steps` steps of one iteration."""
    return [(nk * s // steps, nk * (s + 1) // steps) for s in range(steps)]


def sub_batches(a, b, qmax):
    """[a, b) cut into the fewest nearly equal consecutive batches of at most qmax q."""
    n = b - a
    if n <= 0:
        return []
    m = -(-n // qmax)
    cuts = [a + n * i // m for i in range(m + 1)]
    return [(cuts[i], cuts[i + 1] - cuts[i]) for i in range(m)]


def traffic_record(kernel, tile, precision, cfg_name, path=None):
    """Counter record of `kernel` (HBM bytes per q from FETCH_SIZE / WRITE_SIZE of one launch), or
    None.  Used only for the same workload, precision and tile and an unchanged kernel source."""
    path = path or os.path.join(ROOT, "profiles", f"traffic_{cfg_name.split('_')[0]}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("workload") != cfg_name or rec.get("precision") != precision:
        return None
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
            return None
    k = rec["kernels"].get(kernel)
    if k is None or k["tile"] != tile:
        return None
    return k


# ---------------------------------------------------------------------------------------------
# the CPU oracle on a bounded sample of the same workload
# ---------------------------------------------------------------------------------------------
def cpu_baseline(cfg, prob, budget_s=12.0, R=96):
    import gwinputs as gi
    import oracle as o
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(p.get("num_threads", 1)) for p in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    rows = np.arange(R)
    g = gi.MGenerator(cfg)
    blocks = [g.block(0, k, rows=rows) for k in range(cfg.nk)]
    G = o.green0(prob.eps, prob.nb, prob.tau, cfg.beta)
    done, flops, t_used = [], 0.0, 0.0
    for it in range(prob.tau.size):
        t0 = time.perf_counter()
        o.polarization(blocks, G, prob.kmq[0], cfg.scale, taus=[it])
        t_used += time.perf_counter() - t0
        done.append(it)
        flops += sum(8.0 * R * R * b.shape[1] * b.shape[2] for b in blocks)
        if t_used > budget_s:
            break
    return {"value": flops / t_used / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"the oracle's polarization of q = 0 for I, J < {R}, all {cfg.nk} k, {len(done)} of "
                      f"{prob.tau.size} tau points ({flops:.3e} flop in {t_used:.1f} s; numpy FP64 on "
                      f"{cores} BLAS threads)"}


# ---------------------------------------------------------------------------------------------
# the batching study (one launch vs a per-k launch loop), a mode of its own
# ---------------------------------------------------------------------------------------------
def batching_study(args):
    """One launch over all (k, tau) blocks of a q against one launch per k block, on one q.

    The uneven 6x6x6-k workload (Nb_k in [96, 160], NI_q in [500, 900], 121 tau points) by default,
    on its q with the largest NI; pair-space kernels of the split precision, M resident in HBM.
    Prints one JSON line with both times for the polarization and the self-energy and the relative
    difference of the two results (they differ only in where the FP32 partial sums are flushed)."""
    import torch
    import gwinputs as gi
    import paper_1602_02313_amd as amd

    cfg = gi.CONFIGS[args.config]
    prob = gi.make_problem(cfg)
    q = int(np.argmax(prob.ni))
    B = {"f16x3": amd.F16X3, "bf16x3": amd.BF16X3}[args.precision]
    run = amd.GWRun(cfg.nk, prob.kmq, prob.nb, prob.ni, prob.tau, cfg.beta, cfg.niw_f, cfg.niw_b,
                    cfg.scale, prob.eps, prob.v, prob.n_target, precision=B, q_batch=1)
    M = torch.empty(int(run.mpre[q + 1] - run.mpre[q]), dtype=torch.complex64, device="cuda")
    run.ctx.synth_M(cfg.seed, q, 1, 1, amd.C64, M)
    run.green0(0.0)
    NI, ntau = int(prob.ni[q]), int(prob.tau.size)
    gen = torch.Generator(device="cuda").manual_seed(7)
    W = run.Wt_tau[:ntau * NI * NI]
    W.copy_(torch.randn(W.shape, dtype=torch.complex128, device="cuda", generator=gen) * 1e-3)
    ctx = run.ctx
    fp, fs = flop_model(prob, qs=[q])
    log(f"[batching] {cfg.name} q={q} NI={NI}: M {M.numel() * 8 / 1e9:.1f} GB")

    def timed(fn):
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    def p_one():
        ctx.polarization(q, 1, M, amd.C64, run.G_tau, B, run.P_tau)

    P2 = torch.empty(ntau * NI * NI, dtype=torch.complex128, device="cuda")

    def p_loop():
        for k in range(cfg.nk):
            ctx.set_k_range(k, k + 1, reuse_prepared=k > 0)
            ctx.polarization(q, 1, M, amd.C64, run.G_tau, B, P2)
        ctx.set_k_range()

    def s_one():
        run.sig_tau.zero_()
        ctx.self_energy(q, 1, M, amd.C64, run.G_tau, run.Wt_tau, B, run.sig_tau)

    sig_loop = torch.zeros_like(run.sig_tau)

    def s_loop():
        sig_loop.zero_()
        for k in range(cfg.nk):
            ctx.set_k_range(k, k + 1, reuse_prepared=k > 0)
            ctx.self_energy(q, 1, M, amd.C64, run.G_tau, run.Wt_tau, B, sig_loop)
        ctx.set_k_range()

    res = {}
    for name, one, loop, nfl in (("polarization", p_one, p_loop, fp), ("self_energy", s_one, s_loop, fs)):
        one()
        t1 = min(timed(one) for _ in range(2))
        loop()
        tl = min(timed(loop) for _ in range(2))
        log(f"[batching] {name}: one launch {t1:.1f} ms, {cfg.nk} launches {tl:.1f} ms")
        res[name] = {"one_launch_ms": round(t1, 2), "per_k_loop_ms": round(tl, 2),
                     "calls_in_loop": cfg.nk, "loop_over_one": round(tl / t1, 3),
                     "one_launch_tflops": round(nfl / (t1 / 1e3) / 1e12, 1)}
    n = ntau * NI * NI
    a, b = run.P_tau[:n], P2
    res["polarization"]["loop_vs_one_rel"] = float((a - b).abs().norm() / a.abs().norm())
    a, b = run.sig_tau, sig_loop
    res["self_energy"]["loop_vs_one_rel"] = float((a - b).norm() / a.norm())
    print(json.dumps({"study": "batching: all (k, tau) blocks of a q in one launch vs one launch per k",
                      "workload": f"{cfg.name}, q = {q} (NI = {NI}), {cfg.nk} k blocks with uneven band "
                                  f"counts, {ntau} tau points, {args.precision} pair-space kernels",
                      "unit": "ms", **res}), flush=True)


def queue_study(args):
    """The pair-space polarization of one q batch with a static grid (hardware dispatch of an
    XCD-ordered work list, equal item counts per XCD) against its persistent form (one work-group per CU
    taking items from per-XCD device queues cut by equal cost, items in decreasing cost), on the uneven
    workload: 6x6x6 k, Nb_k in [96, 160], NI_q in [500, 900], q = 0..nq-1 in one call.  Prints one JSON
    line with both times and the difference of the results."""
    import torch
    import gwinputs as gi
    import paper_1602_02313_amd as amd

    cfg = gi.CONFIGS["c4"]
    prob = gi.make_problem(cfg)
    nq = args.q_batch
    B = {"f16x3": amd.F16X3, "bf16x3": amd.BF16X3}[args.precision]
    run = amd.GWRun(cfg.nk, prob.kmq, prob.nb, prob.ni, prob.tau, cfg.beta, cfg.niw_f, cfg.niw_b,
                    cfg.scale, prob.eps, prob.v, prob.n_target, precision=B, q_batch=nq)
    M = torch.empty(int(run.mpre[nq]), dtype=torch.complex64, device="cuda")
    run.ctx.synth_M(cfg.seed, 0, nq, 1, amd.C64, M)
    run.green0(0.0)
    names = run.ctx.variants(amd.OP_POLARIZATION, B)
    vq = next(i for i, n in enumerate(names) if "queue" in n)
    vs = names.index("pair-space 16x16 pairs K64 st4x8 3-buffer")
    fp, _ = flop_model(prob, qs=range(nq))
    log(f"[queue] {cfg.name} q 0..{nq - 1}, NI {list(prob.ni[:nq])}: M {M.numel() * 8 / 1e9:.1f} GB")
    res, outs = {}, {}
    for label, v in (("static_grid", vs), ("persistent_queue", vq)):
        run.ctx.set_variant(amd.OP_POLARIZATION, B, v)
        ts = []
        for rep in range(3):
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            run.ctx.polarization(0, nq, M, amd.C64, run.G_tau, B, run.P_tau)
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
            log(f"[queue] {label} rep {rep}: {ts[-1]:.1f} ms")
        t = min(ts[1:])
        res[label] = {"variant": names[v], "ms": round(t, 1), "dense_tflops": round(fp / (t / 1e3) / 1e12, 1)}
        outs[label] = run.P_tau[: int(run.ppre[nq])].clone()
    a, b = outs["static_grid"], outs["persistent_queue"]
    print(json.dumps({"study": "persistent work queue vs static grid, pair-space polarization of one q batch",
                      "workload": f"{cfg.name}: q 0..{nq - 1} (NI {[int(x) for x in prob.ni[:nq]]}), {cfg.nk} k "
                                  f"blocks with Nb_k in [96, 160], {prob.tau.size} tau points, {args.precision}",
                      **res, "queue_over_static": round(res["persistent_queue"]["ms"] / res["static_grid"]["ms"], 3),
                      "rel_diff": float((a - b).abs().norm() / a.abs().norm())}), flush=True)


def screen_study(args):
    """The FP64 screen (msgw_screen: the inversion of 1 - v^1/2 P v^1/2 and the forming of W~ and R) on
    one call of the iteration's shape: 7 q x Niv matrices of the workload's NI, on a synthetic
    negative-definite Hermitian P(i nu) = -1e-3 X X^H (X complex Gaussian / sqrt(NI)), the same for
    every matrix (so the Hermitian sweep inverts them all).  Times four calls with HIP events and checks the first W~ against numpy's solve of
    (1 - chi) Y = chi, W~ = v^1/2 Y v^1/2.  Prints one JSON line."""
    import numpy as np
    import torch
    import gwinputs as gi
    import paper_1602_02313_amd as amd

    cfg = gi.CONFIGS[args.config]
    prob = gi.make_problem(cfg)
    nq = 7
    run = amd.GWRun(cfg.nk, prob.kmq, prob.nb, prob.ni, prob.tau, cfg.beta, cfg.niw_f, cfg.niw_b, cfg.scale,
                    prob.eps, prob.v, prob.n_target, precision=amd.F16X3, q_batch=nq)
    NI, nw = int(prob.ni[0]), cfg.niw_b
    if any(int(x) != NI for x in prob.ni[:nq]):
        raise SystemExit("the screen study needs equal NI over its q")
    rng = np.random.default_rng(3)
    X = (rng.normal(size=(NI, NI)) + 1j * rng.normal(size=(NI, NI))) / np.sqrt(NI)
    B = -(X @ X.conj().T) * 1e-3
    Piw = torch.from_numpy(np.broadcast_to(B, (nq * nw, NI, NI)).copy().ravel()).to("cuda")
    Wt, R = torch.zeros_like(Piw), torch.zeros_like(Piw)
    info = torch.zeros(nq * nw, dtype=torch.int32, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    v = run.v[: nq * NI]
    log(f"[screen] {cfg.name}: {nq} q x {nw} nu matrices of NI = {NI}")
    ts = []
    for rep in range(4):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        run.ctx.screen(0, nq, Piw, v, Wt, R, info, flags)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
        log(f"[screen] rep {rep}: {ts[-1]:.2f} ms")
    sv = np.sqrt(v[:NI].cpu().numpy())
    chi = sv[:, None] * B * sv[None, :]
    Wr = sv[:, None] * np.linalg.solve(np.eye(NI) - chi, chi) * sv[None, :]
    W0 = Wt[: NI * NI].cpu().numpy().reshape(NI, NI)
    t = min(ts)
    print(json.dumps({"study": "FP64 screen (Hermitian P: blocked sweep; else pivoting Gauss-Jordan) of one q batch",
                      "workload": f"{cfg.name}: {nq} q x {nw} nu = {nq * nw} matrices of NI = {NI}",
                      "ms_per_call": round(t, 2), "s_per_iteration": round(t * cfg.nk / nq / 1e3, 2),
                      "tflops_at_10.7_NI3": round(10.7 * NI ** 3 * nq * nw / (t / 1e3) / 1e12, 1),
                      "rel_err_vs_numpy": float(np.linalg.norm(W0 - Wr) / np.linalg.norm(Wr)),
                      "info": int(info.abs().sum()), "flags": int(flags.item())}), flush=True)


def full_study(args):
    """The FULL band-matrix self-energy in split FP16 against the diagonal one on one q of the 4x4x4 k,
    64-band, NI = 400, 81-tau workload: P, the screen and W~(tau) of q = 0 in FP64 (M drawn on the
    device), then Sigma^c of that q in FULL (k_sf_ywm + k_sf_contract) and in DIAG (k_sigz) mode, both
    F16X3 on the same W~ and M.  The real part of FULL's diagonal is DIAG's Sigma (the DIAG kernels use
    the Hermitian part of W~, the same sum).  Prints one JSON line with both times, their dense-model
    rates and the largest difference."""
    import torch
    import gwinputs as gi
    import paper_1602_02313_amd as amd

    cfg = gi.CONFIGS["c2"]
    prob = gi.make_problem(cfg)
    mk = lambda prec, mode: amd.GWRun(cfg.nk, prob.kmq, prob.nb, prob.ni, prob.tau, cfg.beta, cfg.niw_f,
                                      cfg.niw_b, cfg.scale, prob.eps, prob.v, prob.n_target, precision=prec,
                                      sigma_mode=mode, q_batch=1)
    r64 = mk(amd.FP64, amd.SIGMA_DIAG)
    M64 = torch.empty(int(r64.mpre[1]), dtype=torch.complex128, device="cuda")
    r64.ctx.synth_M(cfg.seed, 0, 1, 1, amd.C128, M64)
    r64.green0(0.0)
    r64.begin_pass()
    r64.q_block(amd.ResidentM(M64, r64.mpre), 0, 1)
    W = r64.Wt_tau[: int(r64.ppre[1])].clone()
    del M64, r64
    torch.cuda.empty_cache()
    log(f"[full] {cfg.name}: W~ of q = 0 in FP64")
    res, out = {}, {}
    for label, mode in (("full", amd.SIGMA_FULL), ("diag", amd.SIGMA_DIAG)):
        run = mk(amd.F16X3, mode)
        M = torch.empty(int(run.mpre[1]), dtype=torch.complex64, device="cuda")
        run.ctx.synth_M(cfg.seed, 0, 1, 1, amd.C64, M)
        run.green0(0.0)
        ts = []
        for rep in range(2):
            run.sig_tau.zero_()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            run.ctx.self_energy(0, 1, M, amd.C64, run.G_tau, W, amd.F16X3, run.sig_tau)
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
            log(f"[full] {label} rep {rep}: {ts[-1]:.1f} ms")
        out[label] = run.sig_tau.clone()
        res[label] = {"ms": round(min(ts), 1)}
        del run, M
        torch.cuda.empty_cache()
    ntau = prob.tau.size
    ni = int(prob.ni[0])
    f_full = f_diag = 0.0
    for k in range(cfg.nk):
        nn, nm = int(prob.nb[k]), int(prob.nb[prob.kmq[0, k]])
        f_diag += 8.0 * ni * ni * nn * nm * ntau + 8.0 * ni * nn * nm * ntau
        f_full += 8.0 * ni * ni * nn * nm * ntau + 8.0 * ni * nn * nn * nm * ntau
    res["full"]["dense_tflops"] = round(f_full / (res["full"]["ms"] / 1e3) / 1e12, 1)
    res["diag"]["dense_tflops"] = round(f_diag / (res["diag"]["ms"] / 1e3) / 1e12, 1)
    diag_of_full = torch.diagonal(out["full"], dim1=1, dim2=2).real.permute(0, 2, 1)
    d = out["diag"]
    print(json.dumps({"study": "FULL band-matrix Sigma^c vs DIAG in split FP16, one q",
                      "workload": f"{cfg.name}: q = 0, {cfg.nk} k blocks of {int(prob.nb[0])} bands, NI = {ni}, "
                                  f"{ntau} tau points, W~ from the FP64 chain",
                      **res, "full_over_diag": round(res["full"]["ms"] / res["diag"]["ms"], 2),
                      "rel_diff_re_diag_full_vs_diag": float((diag_of_full - d).norm() / d.norm())}), flush=True)


def tau_solver_study(args):
    """The paper's tau-domain solvers against the Matsubara-axis route on the same inputs, FP64:
    W~(q, tau) of 4 q from the linear system of order 81 x 50 = 4050 (the 4x4x4-k workload's 81-point
    UPM mesh, beta = 200, NI = 50 so that the system fits the 4096 limit; P from the library's FP64
    polarization on M drawn on the device) against P(tau) -> P(i nu) -> screen -> W~(tau), with the
    workload's Coulomb matrix and with it scaled by 1e-5; and G(k, tau)
    of the states of 2 k from the Dyson equation on the dense uniform grid (an 81-point UPM mesh at
    beta = 50: 1281 dense points, one system of order 1281 per state) against Sigma(i w) -> Dyson on i w
    -> G(tau), at a fixed mu, for a synthetic Sigma^c(tau) of two fermionic poles per state and a static
    shift.  Both tau routes call the library's host-synchronous entry points; the times are wall
    clock around them (the i nu routes with a device synchronization).  Prints one JSON line."""
    import torch
    import gwinputs as gi
    import paper_1602_02313_amd as amd

    out = {}
    # the W~ system
    cfg = gi.CONFIGS["c2"].replace(name="c2_ni50", ni=50, grid=(2, 2, 1))
    prob = gi.make_problem(cfg)
    nq = 4
    run = amd.GWRun(cfg.nk, prob.kmq, prob.nb, prob.ni, prob.tau, cfg.beta, cfg.niw_f, cfg.niw_b, cfg.scale,
                    prob.eps, prob.v, prob.n_target, precision=amd.FP64, q_batch=nq)
    M = torch.empty(int(run.mpre[nq]), dtype=torch.complex128, device="cuda")
    run.ctx.synth_M(cfg.seed, 0, nq, 1, amd.C128, M)
    run.green0(0.0)
    run.ctx.polarization(0, nq, M, amd.C128, run.G_tau, amd.FP64, run.P_tau)
    NI, nt = int(prob.ni[0]), prob.tau.size
    nbytes = run.ctx.tau_solver_work_size(amd.TS_WTILDE, 0, nq)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    info = torch.zeros(nq, dtype=torch.int32, device="cuda")
    Wsys = torch.zeros(nq * nt * NI * NI, dtype=torch.complex128, device="cuda")
    out["w_tilde"] = {"shape": f"{nq} q, {nt} tau points, NI = {NI}: systems of order {nt * NI} with {NI} "
                               f"right-hand sides"}
    # the workload's Coulomb matrix, whose screening is far faster than the mesh spacing at tau = 0, and
    # the same scaled by 1e-5 (largest eigenvalue of v^1/2 P(0) v^1/2 of order 1), where the mesh
    # resolves W~(tau)
    for label, f in (("coulomb", 1.0), ("coulomb_x1e-5", 1e-5)):
        v = (run.v[: nq * NI] * f).contiguous()
        tnu, tsys = [], []
        for rep in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run.ctx.tau_to_iw(amd.BOSON, nq, NI * NI, run.P_tau, 1, None, run.P_iw)
            run.ctx.screen(0, nq, run.P_iw, v, run.Wt_iw, run.R_iw, run.info, run.screen_flags)
            run.ctx.screened_tau(0, nq, run.R_iw, run.P_tau, v, run.Wt_tau)
            torch.cuda.synchronize()
            tnu.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            run.ctx.wt_tau_system(0, nq, run.P_tau, v, Wsys, info, work, nbytes)
            torch.cuda.synchronize()
            tsys.append(time.perf_counter() - t0)
            log(f"[tau] W~ ({label}): nu route {tnu[-1] * 1e3:.1f} ms, tau system {tsys[-1] * 1e3:.1f} ms")
        Wnu = run.Wt_tau[: nq * nt * NI * NI]
        out["w_tilde"][label] = {"nu_route_ms": round(1e3 * min(tnu[1:]), 2),
                                 "tau_system_ms": round(1e3 * min(tsys[1:]), 2), "info": int(info.abs().max()),
                                 "max_diff_over_max": float((Wsys - Wnu).abs().max() / Wnu.abs().max())}
    del run, M, work, Wsys
    torch.cuda.empty_cache()
    # the G Dyson on the dense grid
    cfg = gi.Config(name="dys_upm81", grid=(2, 1, 1), bands=((4, -1.0, -0.2), (4, 0.1, 1.5)), nb=None, ni=6,
                    nb_range=(4, 8), ntau=80, mesh="upm", beta=50.0, niw_f=256, niw_b=16)
    prob = gi.make_problem(cfg)
    run = amd.GWRun(cfg.nk, prob.kmq, prob.nb, prob.ni, prob.tau, cfg.beta, cfg.niw_f, cfg.niw_b, cfg.scale,
                    prob.eps, prob.v, prob.n_target, precision=amd.FP64, q_batch=1)
    rng = np.random.default_rng(5)
    nk, nbmax, nt, beta = cfg.nk, prob.eps.shape[1], prob.tau.size, cfg.beta

    def g0(e, tau):  # -e^{-e tau} / (1 + e^{-beta e}) in its overflow-free form
        return -np.exp(-e * tau) / (1.0 + np.exp(-beta * e)) if e >= 0 else \
            -np.exp(e * (beta - tau)) / (1.0 + np.exp(beta * e))
    sig = np.zeros((nk, nbmax, nt))
    sst = np.zeros((nk, nbmax))
    for k in range(nk):
        for n in range(int(prob.nb[k])):
            for _ in range(2):
                sig[k, n] += rng.uniform(0.01, 0.05) * g0(rng.uniform(-1.0, 1.0), prob.tau)
            sst[k, n] = rng.uniform(-0.1, 0.1)
    mu = 0.05
    run.sig_tau.copy_(torch.from_numpy(sig))
    run.sig_x.copy_(torch.from_numpy(sst))
    nbytes = run.ctx.tau_solver_work_size(amd.TS_DYSON, 0, nk)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    Gt = torch.zeros((nk, nbmax, nt), dtype=torch.float64, device="cuda")
    info = torch.zeros(nk * nbmax, dtype=torch.int32, device="cuda")
    tnu, tsys = [], []
    for rep in range(3):
        run.mu.fill_(mu)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run.sigma_to_iw()
        run._dyson(search=False)
        torch.cuda.synchronize()
        tnu.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        run.ctx.dyson_tau(0, nk, run.eps, run.sig_x, run.mu, run.sig_tau, Gt, info, work, nbytes)
        torch.cuda.synchronize()
        tsys.append(time.perf_counter() - t0)
        log(f"[tau] G: i w route {tnu[-1] * 1e3:.1f} ms, dense-grid Dyson {tsys[-1] * 1e3:.1f} ms")
    nstates = int(sum(int(x) for x in prob.nb))
    out["dyson"] = {"shape": f"{nstates} states on {nk} k, {nt} tau points (UPM, beta = {beta:g}), dense grid of "
                             f"{int(round(beta / (prob.tau[1] - prob.tau[0]))) + 1} points",
                    "iw_route_ms": round(1e3 * min(tnu[1:]), 2), "tau_dyson_ms": round(1e3 * min(tsys[1:]), 2),
                    "info": int(info.abs().max()),
                    "max_abs_diff": float((Gt - run.G_tau).abs().max())}
    print(json.dumps({"study": "the paper's tau-domain solvers against the Matsubara-axis route, FP64", **out}),
          flush=True)


def symmetry_study(args):
    """One self-energy pass plus Dyson and gap over the full zone against the irreducible-wedge pass
    (P, W~ and the contractions for the irreducible q only, contributions added over the stars), on
    the metric's workload shapes with the symmetry of a cubic crystal: 5x5x5 k, 128 bands, NI = 691
    (the closed shells of |G|^2 <= 29, the nearest to 700), 161 tau points, M generated on the device
    per q (msgw_synth_M_cubic).  Prints one JSON line with both times and the difference of the results."""
    import torch
    import gwinputs as gi
    import paper_1602_02313_amd as amd
    from paper_1602_02313_amd.driver import EventTimer

    base = gi.CONFIGS[args.config]
    cfg = base.replace(name=base.name + "_cubic", ni=691)
    prob = gi.make_cubic_problem(cfg)
    prec = {"f16x3": amd.F16X3, "bf16x3": amd.BF16X3, "fp32": amd.FP32, "fp64": amd.FP64}[args.precision]
    rot_k = gi.rotation_k_maps(cfg)
    gen = amd.SynthCubicM(cfg.seed)
    t_start = time.time()

    def src(run, q0, nq):  # the device generator, with a progress line per q block (the wait costs ~0.1 ms)
        torch.cuda.synchronize()
        log(f"[symmetry] q {q0}..{q0 + nq - 1} at {time.time() - t_start:.0f} s")
        return gen(run, q0, nq)

    out = {}
    results = {}
    for mode in ("ibz", "full"):
        run = amd.GWRun(cfg.nk, prob.kmq, prob.nb, prob.ni, prob.tau, cfg.beta, cfg.niw_f, cfg.niw_b,
                        cfg.scale, prob.eps, prob.v, prob.n_target, precision=prec,
                        q_batch=1 if mode == "ibz" else args.q_batch)
        if mode == "ibz":
            run.set_symmetry(rot_k)
        run.green0(0.0)
        torch.cuda.synchronize()
        t = EventTimer()
        run.timer = t
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        run.sigma_pass(src)
        run.dyson(True)
        run.gap()
        b.record()
        torch.cuda.synchronize()
        run.timer = None
        sec = a.elapsed_time(b) / 1e3
        nq = len(run.ibz) if mode == "ibz" else cfg.nk
        log(f"[symmetry] {mode}: {nq} q, {sec:.1f} s")
        out[mode] = {"q": nq, "s_per_iteration": round(sec, 2),
                     "contraction_s": round(sum(sum(v) for k, v in t.summary().items()
                                                if k in ("polarization", "self_energy")) / 1e3, 2)}
        results[mode] = (run.sig_tau.clone(), run.sig_x.clone(), float(run.gap_d.item()), run.flags.item())
        del run
        torch.cuda.empty_cache()
    (si, xi, gi_, fi), (sf, xf, gf, ff) = results["ibz"], results["full"]
    print(json.dumps({
        "study": "crystal symmetry: irreducible q with their stars vs the full zone (one iteration)",
        "workload": f"{cfg.name}: 5x5x5 k, 128 bands, NI = 691, {prob.tau.size} tau points, {args.precision}",
        "full_zone": out["full"], "irreducible_wedge": out["ibz"],
        "speedup": round(out["full"]["s_per_iteration"] / out["ibz"]["s_per_iteration"], 2),
        "sigma_c_rel_diff": float((si - sf).norm() / sf.norm()),
        "sigma_x_rel_diff": float((xi - xf).norm() / xf.norm()),
        "gap_diff_Ha": abs(gi_ - gf), "flags": int(fi) | int(ff)}), flush=True)


# ---------------------------------------------------------------------------------------------
# the FP64 GPU path on a subset of the same inputs
# ---------------------------------------------------------------------------------------------
def fp64_reference(cfg, prob, kref):
    import torch
    import paper_1602_02313_amd as amd
    from paper_1602_02313_amd.driver import EventTimer
    ref = amd.GWRun(cfg.nk, prob.kmq, prob.nb, prob.ni, prob.tau, cfg.beta, cfg.niw_f, cfg.niw_b,
                    cfg.scale, prob.eps, prob.v, prob.n_target, precision=amd.FP64, q_batch=1)
    M64 = torch.empty(int(ref.mpre[1]), dtype=torch.complex128, device="cuda")
    ref.ctx.synth_M(cfg.seed, 0, 1, 1, amd.C128, M64)
    ref.green0(0.0)
    kref = min(kref, cfg.nk)
    ref.ctx.set_k_range(0, kref)
    src = amd.ResidentM(M64, ref.mpre)
    ref.begin_pass()
    ref.q_block(src, 0, 1)      # warm-up
    t64 = EventTimer(ctx=ref.ctx)
    ref.timer = t64
    ref.begin_pass()
    ref.q_block(src, 0, 1)
    ref.timer = None
    k64 = t64.kernel_summary()
    ref.ctx.set_k_range()
    fp1, fs1 = flop_model(prob, qs=[0], ks=range(kref))
    tp, ts = k64["polarization"][0] / 1e3, k64["self_energy"][0] / 1e3
    out = {"subset": f"q = 0, k blocks 0..{kref - 1} of {cfg.nk} (the workload's block shapes)",
           "polarization_tflops": round(fp1 / tp / 1e12, 2), "self_energy_tflops": round(fs1 / ts / 1e12, 2),
           "p_plus_sigma_tflops": round((fp1 + fs1) / (tp + ts) / 1e12, 2), "peak": PEAK["fp64"],
           "p_plus_sigma_s_per_iteration_at_this_rate": None}
    del M64, ref
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c5")
    ap.add_argument("--precision", default="f16x3", choices=["f16x3", "bf16x3", "fp32", "fp64"])
    ap.add_argument("--q-batch", type=int, default=8, help="largest q batch of one library call")
    ap.add_argument("--fp64-ref-k", type=int, default=4,
                    help="k blocks of q = 0 on which the FP64 GPU path is timed for comparison (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--variant-p", type=int, default=None,
                    help="polarization tile variant (skips the autotuner for P)")
    ap.add_argument("--variant-s", type=int, default=None,
                    help="self-energy tile variant (skips the autotuner for Sigma)")
    ap.add_argument("--profile-batch", action="store_true",
                    help="counter runs: a plain device copy of --copy-mb MB, then the first q batch of the "
                         "path, no timing and no JSON line")
    ap.add_argument("--copy-mb", type=int, default=1024)
    ap.add_argument("--graph", action="store_true",
                    help="each step captured once as a HIP graph and replayed (no per-kernel times)")
    ap.add_argument("--queue", action="store_true",
                    help="instead of the iteration: static grid vs persistent work queue for the polarization "
                         "of one --q-batch of the uneven workload")
    ap.add_argument("--symmetry", action="store_true",
                    help="instead of the iteration: full zone vs irreducible wedge on the cubic-symmetric "
                         "form of --config (NI = 691)")
    ap.add_argument("--tau-solvers", action="store_true",
                    help="instead of the iteration: the tau-domain W~ system and G Dyson against the i nu / i w routes")
    ap.add_argument("--full", action="store_true",
                    help="instead of the iteration: FULL vs DIAG split-FP16 self-energy on one q of c2")
    ap.add_argument("--screen", action="store_true",
                    help="instead of the iteration: time the FP64 screen on one 7-q call of --config")
    ap.add_argument("--batching", action="store_true",
                    help="instead of the iteration: one launch vs a per-k launch loop on one q of --config "
                         "(default c4, the uneven workload)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): there is no multi-GPU path; "
              f"it would shard the q axis over GPUs with one all-reduce of Sigma per iteration, which is "
              f"not implemented", file=sys.stderr)
        sys.exit(2)
    if args.symmetry:
        symmetry_study(args)
        return
    if args.queue:
        queue_study(args)
        return
    if args.screen:
        screen_study(args)
        return
    if args.full:
        full_study(args)
        return
    if args.tau_solvers:
        tau_solver_study(args)
        return
    if args.batching:
        if args.config == "c5":
            args.config = "c4"
        batching_study(args)
        return

    import torch
    import gwinputs as gi
    import paper_1602_02313_amd as amd
    from paper_1602_02313_amd.driver import EventTimer

    cfg = gi.CONFIGS[args.config]
    prob = gi.make_problem(cfg)
    prec = {"f16x3": amd.F16X3, "bf16x3": amd.BF16X3, "fp32": amd.FP32, "fp64": amd.FP64}[args.precision]
    steps = max(1, min(args.steps, cfg.nk))
    slices = iteration_slices(cfg.nk, steps)
    qb = max(1, min(args.q_batch, max(b - a for a, b in slices)))
    log(f"[bench] {cfg.name}: nk={cfg.nk} nb={int(prob.nb.max())} NI={int(prob.ni.max())} "
        f"ntau={prob.tau.size} niw={cfg.niw_f} precision={args.precision}; {steps} steps of "
        f"{min(b - a for a, b in slices)}-{max(b - a for a, b in slices)} q per iteration, q batch {qb}")
    run = amd.GWRun(cfg.nk, prob.kmq, prob.nb, prob.ni, prob.tau, cfg.beta, cfg.niw_f, cfg.niw_b,
                    cfg.scale, prob.eps, prob.v, prob.n_target, precision=prec, q_batch=qb)
    src = amd.SynthM(cfg.seed, symmetric=True)
    src.reserve(run)
    fixed = {amd.OP_POLARIZATION: args.variant_p, amd.OP_SELF_ENERGY: args.variant_s}
    for op, v in fixed.items():
        if v is not None:
            run.ctx.set_variant(op, prec, v)
    if args.profile_batch:
        # a plain copy of known size calibrates the HBM byte counters, then one q batch of the path
        n = args.copy_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        run.green0(0.0)
        run.begin_pass()
        run.q_block(src, 0, qb)
        torch.cuda.synchronize()
        vp = run.ctx.get_variant(amd.OP_POLARIZATION, prec)
        vs = run.ctx.get_variant(amd.OP_SELF_ENERGY, prec)
        log(f"[bench] profile batch done: copy of {args.copy_mb} MB, q 0..{qb - 1}, variants "
            f"P {vp} ({run.ctx.variants(amd.OP_POLARIZATION, prec)[vp]}) "
            f"S {vs} ({run.ctx.variants(amd.OP_SELF_ENERGY, prec)[vs]})")
        return
    tuned = {}
    if not args.no_autotune and prec != amd.FP64 and None in fixed.values():
        from paper_1602_02313_amd import autotune
        ops = [op for op, v in fixed.items() if v is None]
        for op, (v, name, times) in autotune.tune(run, src, reps=1, log=log, ops=ops, nq=1).items():
            tuned[["polarization", "self_energy"][op]] = {"variant": v, "tile": name, "ms": times}

    run.green0(0.0)
    run.mu.zero_()

    def step(s):
        a, b = slices[s]
        if s == 0:
            run.begin_pass()
        for q0, nq in sub_batches(a, b, qb):
            run.q_block(src, q0, nq)
        if s == steps - 1:
            run.sigma_to_iw()
            run.dyson(True)
            run.gap()

    graphs = None
    if args.graph:
        torch.cuda.synchronize()
        graphs = []
        for s in range(steps):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                step(s)
            graphs.append(g)
        torch.cuda.synchronize()
        run.green0(0.0)
        run.mu.zero_()

    def do(s):
        if graphs is not None:
            graphs[s].replay()
        else:
            step(s)

    t0 = time.perf_counter()
    for w in range(args.warmup):
        do(w % steps)
        torch.cuda.synchronize()
        log(f"[bench] warmup {w} (q {slices[w % steps][0]}..{slices[w % steps][1] - 1}) done at "
            f"{time.perf_counter() - t0:.2f} s")
    timer = EventTimer(ctx=run.ctx)
    run.timer = None if graphs is not None else timer
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        do(s)
        torch.cuda.synchronize()
        log(f"[bench] step {s} (q {slices[s][0]}..{slices[s][1] - 1}) done at {time.perf_counter() - t0:.2f} s")
    t_tot = time.perf_counter() - t0
    run.timer = None
    ms_step = 1e3 * t_tot / steps
    flags = int(run.flags.item()) | int(run.screen_flags.item())
    gap, N, mu = float(run.gap_d.item()), float(run.N.item()), float(run.mu.item())
    fp, fs = flop_model(prob)
    value = (fp + fs) / (t_tot) / 1e12

    line_extra = {}
    roof = None
    kernels = None
    if graphs is None:
        kern = timer.summary()
        kk = timer.kernel_summary()
        ksum = {k: float(np.sum(v)) for k, v in kern.items()}
        dom = max(("polarization", "self_energy"), key=lambda k: ksum.get(k, 0.0))
        op = {"polarization": amd.OP_POLARIZATION, "self_energy": amd.OP_SELF_ENERGY}[dom]
        tile = run.ctx.variants(op, prec)[run.ctx.get_variant(op, prec)] if prec != amd.FP64 else "fp64"
        calls = [(q0, nq) for a, b in slices for q0, nq in sub_batches(a, b, qb)]
        ktimes = kk[dom]
        assert len(ktimes) == len(calls), (len(ktimes), len(calls))
        exe = [executed_mfma_flops(prob, op, tile, q0, nq) for q0, nq in calls]
        dense = [flop_model(prob, qs=range(q0, q0 + nq))[op] for q0, nq in calls]
        t_k = float(np.sum(ktimes)) / 1e3
        avg_ms = float(np.mean(ktimes))
        if exe[0] is not None and args.precision in ("f16x3", "bf16x3"):
            achieved = float(np.sum(exe)) / t_k / 1e12
            roof = {"bound": "mfma", "achieved": round(achieved, 1), "peak": PEAK_16, "unit": "TFLOP/s",
                    "frac": round(achieved / PEAK_16, 4)}
        else:
            achieved = float(np.sum(dense)) / t_k / 1e12
            roof = {"bound": "mfma", "achieved": round(achieved, 1), "peak": PEAK[args.precision],
                    "unit": "TFLOP/s", "frac": round(achieved / PEAK[args.precision], 4)}
        rec = traffic_record(dom, tile, args.precision, cfg.name)
        qavg = float(np.mean([nq for _, nq in calls]))
        roof.update({
            "traffic": round(rec["bytes_per_q"] * qavg) if rec else None,
            "kernel": {"polarization": "k_polz", "self_energy": "k_sigz"}[dom] if exe[0] is not None else dom,
            "tile": tile,
            "avg_launch_ms": round(avg_ms, 2),
            "launches": len(ktimes),
            "executed_flop_per_launch": round(float(np.mean(exe))) if exe[0] is not None else None,
            "dense_equiv_tflops": round(float(np.sum(dense)) / t_k / 1e12, 1),
            "basis": ("achieved = MFMA flops the kernel executes (counted from its loops: Hermitian "
                      "triangle, real weight against complex pair products, tile padding) over its "
                      "event-timed duration, against the dense 16-bit MFMA peak; dense_equiv_tflops = "
                      "the dense complex flop model over the same time"),
        })
        kernels = {}
        for k, v in kern.items():
            kernels[k] = {"ms_per_iteration": round(float(np.sum(v)), 1), "calls": len(v)}
            if k in kk:
                kernels[k]["kernel_ms_per_iteration"] = round(float(np.sum(kk[k])), 1)
        kernels["polarization"]["dense_tflops"] = round(fp / (ksum["polarization"] / 1e3) / 1e12, 1)
        kernels["self_energy"]["dense_tflops"] = round(fs / (ksum["self_energy"] / 1e3) / 1e12, 1)

    del src
    run.timer = None
    fp64_ref = None
    if args.fp64_ref_k > 0 and args.precision != "fp64":
        del run
        torch.cuda.empty_cache()
        fp64_ref = fp64_reference(cfg, prob, args.fp64_ref_k)
        fp64_ref["p_plus_sigma_s_per_iteration_at_this_rate"] = round(
            (fp + fs) / (fp64_ref["p_plus_sigma_tflops"] * 1e12), 1)
    cpu = None if args.no_cpu_baseline else cpu_baseline(cfg, prob)

    line = {
        "metric": "P+Sigma effective TFLOP/s and s per scGW iteration, split-FP32 vs FP64 GPU",
        "value": round(value, 2),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 2),
        "s_per_iteration": round(t_tot, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f16x3": "f16x3 (split fp32 on f16 MFMA, scaled operands, fp32 accumulate) + f64",
                  "bf16x3": "bf16x3 (split fp32 on bf16 MFMA, fp32 accumulate) + f64",
                  "fp32": "f32 MFMA + f64", "fp64": "f64"}[args.precision],
        "data": "synthetic (seeded Philox matrix elements drawn on the device per q, model bands, "
                "diagonal Coulomb kernel)",
        "config": {"workload": f"{cfg.name}: one scGW iteration (P, W~, Sigma for all {cfg.nk} q with M "
                               f"generated per q, Dyson with the mu search, gap) in {steps} steps of "
                               f"consecutive q slices",
                   "nk": cfg.nk, "nb": int(prob.nb.max()), "ni": int(prob.ni.max()),
                   "ntau": int(prob.tau.size), "niw_f": cfg.niw_f, "niw_b": cfg.niw_b,
                   "beta": cfg.beta, "precision": args.precision, "q_batch": qb,
                   "hip_graph": bool(args.graph), "flops_p": fp, "flops_sigma": fs},
        "roofline": roof,
        "kernels": kernels,
        "fp64_gpu_reference": fp64_ref,
        "cpu_baseline": cpu,
        "autotune": tuned,
        "check": {"flags": flags, "N": N, "n_target": prob.n_target, "mu": mu, "gap_Ha": gap},
        **line_extra,
    }
    print(json.dumps(line), flush=True)
    if flags:
        log(f"[bench] the iteration raised status flags {flags} (MSGW_FLAG_*): the result is not valid")
        sys.exit(1)


if __name__ == "__main__":
    main()
