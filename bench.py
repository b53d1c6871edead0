#!/usr/bin/env python3
"""Benchmark of the Matsubara-time GW hot path on one MI355X.

A step is one full pass of the path over the 4x4x4 k-grid, 64-band, NI = 400,
81-point UPM workload: G0 -> P(q,tau) -> P(q,i nu) -> W~(q,i nu) -> W~(q,tau) ->
Sigma^c(k,tau), Sigma^x -> Sigma^c(k,i omega) -> Dyson with the mu search -> gap
proxy, for all 64 q.  The inputs (energies, tau mesh, Coulomb kernel and the
complex matrix elements M for every q, 54 GB in complex64) are resident in HBM
before the timed region; M is drawn on the device by the library's Philox
generator.  The metric is the P + Sigma effective TFLOP/s (dense complex flop
model, 8 real flops per complex multiply-add) over the whole step.

    python bench.py [--steps K] [--warmup W] [--precision bf16x3|fp32|fp64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# dense MFMA peaks of MI355X (TFLOP/s).  A split-BF16 product costs three BF16 products, so its
# effective FP32-equivalent peak is the BF16 peak / 3.
PEAK_BF16 = 2516.6
PEAK = {"bf16x3": PEAK_BF16 / 3.0, "f16x3": PEAK_BF16 / 3.0, "fp32": 157.3, "fp64": 78.6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flop_model(prob):
    """Dense complex flop counts of P and Sigma^c (DIAG) for all q."""
    cfg = prob.cfg
    ntau = prob.tau.size
    fp = fs = 0.0
    for q in range(cfg.nk):
        for k in range(cfg.nk):
            nn, nm = int(prob.nb[k]), int(prob.nb[prob.kmq[q, k]])
            ni = int(prob.ni[q])
            fp += 8.0 * ni * ni * nn * nm * ntau
            fs += 8.0 * ni * ni * nn * nm * ntau + 8.0 * ni * nn * nm * ntau
    return fp, fs


def measured_record(kernel, tile, precision, cfg_name, q_batch):
    """Counter record of one launch of `kernel` (HBM bytes, executed MFMA work), or None.

    The record (profiles/traffic_c2_bf16x3.json) holds FETCH_SIZE and WRITE_SIZE of one launch over
    its q_batch q, scaled by a plain copy of known size, together with the SHA-256 of the kernel source
    it was taken on; it is used only for the same workload, precision, q batch, tile and unchanged
    source.
    """
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_c2_bf16x3.json")
    if precision != "bf16x3" or not cfg_name.startswith("c2_") or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("q_batch") != q_batch:
        return None
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
            return None
    k = rec["kernels"].get(kernel)
    if k is None or k["tile"] != tile:
        return None
    return k


def cpu_baseline(cfg, prob, budget_s=12.0):
    """The FP64 oracle's polarization on a bounded sample of the same workload (host cores)."""
    import gwinputs as gi
    import oracle as o
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(p.get("num_threads", 1)) for p in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    R = 160
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
            "sample": f"polarization of q=0, I,J < {R}, all 64 k, {len(done)} of {prob.tau.size} tau "
                      f"points ({flops:.3e} flop in {t_used:.1f} s); numpy FP64 with "
                      f"{cores} BLAS threads"}


def batching_study(args):
    """One launch over all (k, tau) blocks of a q against one launch per k block, on one q.

    The uneven 6x6x6-k workload (Nb_k in [96, 160], NI_q in [500, 900], 121 tau points) by default,
    on its q with the largest NI; split-BF16 pair-space kernels, M resident in HBM.  Prints one JSON
    line with both times for the polarization and the self-energy and the relative difference of the
    two results (they differ only in where the FP32 partial sums are flushed to FP64).
    """
    import torch
    import gwinputs as gi
    import paper_1602_02313_amd as amd

    cfg = gi.CONFIGS[args.config]
    prob = gi.make_problem(cfg)
    q = int(np.argmax(prob.ni))
    run = amd.GWRun(cfg.nk, prob.kmq, prob.nb, prob.ni, prob.tau, cfg.beta, cfg.niw_f, cfg.niw_b,
                    cfg.scale, prob.eps, prob.v, prob.n_target, precision=amd.BF16X3, q_batch=1)
    M = torch.empty(int(run.mpre[q + 1] - run.mpre[q]), dtype=torch.complex64, device="cuda")
    run.ctx.synth_M(cfg.seed, q, 1, 1, amd.C64, M)
    run.green0(0.0)
    NI, ntau = int(prob.ni[q]), int(prob.tau.size)
    gen = torch.Generator(device="cuda").manual_seed(7)
    W = run.Wt_tau[:ntau * NI * NI]
    W.copy_(torch.randn(W.shape, dtype=torch.complex128, device="cuda", generator=gen) * 1e-3)
    ctx, B = run.ctx, amd.BF16X3
    fp, fs = 0.0, 0.0
    for k in range(cfg.nk):
        kk = int(prob.nb[k]) * int(prob.nb[prob.kmq[q, k]])
        fp += 8.0 * NI * NI * kk * ntau
        fs += 8.0 * NI * NI * kk * ntau + 8.0 * NI * kk * ntau
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
                                  f"counts, {ntau} tau points, split-BF16 pair-space kernels",
                      "unit": "ms", **res}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--precision", default="f16x3", choices=["f16x3", "bf16x3", "fp32", "fp64"])
    ap.add_argument("--q-batch", type=int, default=16)
    ap.add_argument("--fp64-ref-q", type=int, default=1,
                    help="q points on which the FP64 GPU path is timed for comparison (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--variant-p", type=int, default=None,
                    help="polarization tile variant (skips the autotuner for P)")
    ap.add_argument("--variant-s", type=int, default=None,
                    help="self-energy tile variant (skips the autotuner for Sigma)")
    ap.add_argument("--profile-batch", action="store_true",
                    help="counter runs: a plain device copy of --copy-mb MB, then one q batch of the path, "
                         "no timing and no JSON line")
    ap.add_argument("--copy-mb", type=int, default=1024)
    ap.add_argument("--graph", action="store_true",
                    help="time replays of the iteration captured as a HIP graph (no per-kernel times)")
    ap.add_argument("--tau-mirror", action="store_true",
                    help="use P(tau) = P(beta - tau) of the symmetric inputs (the dense flop count of the "
                         "metric is unchanged; the saving is reported as tau_mirror in config)")
    ap.add_argument("--batching", action="store_true",
                    help="instead of the pass: one launch vs a per-k launch loop on one q of --config "
                         "(default c4, the uneven workload)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): there is no "
              f"multi-GPU path; it would shard the q axis over GPUs with one all-reduce of Sigma "
              f"per iteration, which is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.batching:
        if args.config == "c2":
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
    log(f"[bench] {cfg.name}: nk={cfg.nk} nb={int(prob.nb.max())} NI={int(prob.ni.max())} "
        f"ntau={prob.tau.size} niw={cfg.niw_f} precision={args.precision}")
    run = amd.GWRun(cfg.nk, prob.kmq, prob.nb, prob.ni, prob.tau, cfg.beta, cfg.niw_f, cfg.niw_b,
                    cfg.scale, prob.eps, prob.v, prob.n_target, precision=prec,
                    q_batch=args.q_batch, tau_mirror=args.tau_mirror)
    ct = torch.complex128 if run.m_dtype == amd.C128 else torch.complex64
    M = torch.empty(int(run.mpre[-1]), dtype=ct, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.ctx.synth_M(cfg.seed, 0, cfg.nk, 1, run.m_dtype, M)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    log(f"[bench] M resident: {M.numel() * M.element_size() / 1e9:.1f} GB generated in {t_gen:.2f} s")
    src = amd.ResidentM(M, run.mpre)
    fixed = {amd.OP_POLARIZATION: args.variant_p, amd.OP_SELF_ENERGY: args.variant_s}
    for op, v in fixed.items():
        if v is not None:
            run.ctx.set_variant(op, prec, v)
    if args.profile_batch:
        # a plain copy of known size calibrates the HBM byte counters, then one batch of the path
        n = args.copy_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        run.green0(0.0)
        run.sig_tau.zero_()
        run.sig_x.zero_()
        run.q_block(src, 0, min(args.q_batch, cfg.nk))
        torch.cuda.synchronize()
        vp = run.ctx.get_variant(amd.OP_POLARIZATION, prec)
        vs = run.ctx.get_variant(amd.OP_SELF_ENERGY, prec)
        log(f"[bench] profile batch done: copy of {args.copy_mb} MB, q 0..{args.q_batch - 1}, variants "
            f"P {vp} ({run.ctx.variants(amd.OP_POLARIZATION, prec)[vp]}) "
            f"S {vs} ({run.ctx.variants(amd.OP_SELF_ENERGY, prec)[vs]})")
        return
    tuned = {}
    if not args.no_autotune and None in fixed.values():
        from paper_1602_02313_amd import autotune
        ops = [op for op, v in fixed.items() if v is None]
        for op, (v, name, times) in autotune.tune(run, src, reps=1, log=log, ops=ops).items():
            tuned[["polarization", "self_energy"][op]] = {"variant": v, "tile": name, "ms": times}

    def step_eager():
        run.green0(0.0)
        run.mu.zero_()
        run.iteration(src)

    step = step_eager
    if args.graph:
        # one pass = G0 + the captured iteration (Sigma pass, Dyson with the mu search, gap)
        graph = run.capture_iteration(src)

        def step():
            run.green0(0.0)
            run.mu.zero_()
            graph.replay()

    for w in range(args.warmup):
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup {w}: {time.perf_counter() - t0:.2f} s")
    timer = EventTimer()
    run.timer = None if args.graph else timer
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step()
        torch.cuda.synchronize()
        log(f"[bench] step {s} done at {time.perf_counter() - t0:.2f} s")
    t_tot = time.perf_counter() - t0
    run.timer = None
    ms_step = 1e3 * t_tot / args.steps
    kern_steps = args.steps
    if args.graph:
        # per-kernel times come from one extra eager pass (kernels cannot be timed inside a replay)
        run.timer = timer
        step_eager()
        torch.cuda.synchronize()
        run.timer = None
        kern_steps = 1
    kern = timer.summary()
    fp, fs = flop_model(prob)
    value = (fp + fs) / (ms_step / 1e3) / 1e12
    flags, gap, N = int(run.flags.item()), float(run.gap_d.item()), float(run.N.item())

    # per-kernel times and the dominant contraction's roofline
    nb_q = -(-cfg.nk // args.q_batch)
    ksum = {k: float(np.sum(v)) / kern_steps for k, v in kern.items()}
    kavg = {k: float(np.mean(v)) for k, v in kern.items()}
    per_launch = {"polarization": fp / nb_q, "self_energy": fs / nb_q}
    dom_op = {"polarization": amd.OP_POLARIZATION, "self_energy": amd.OP_SELF_ENERGY}
    dom = max(("polarization", "self_energy"), key=lambda k: ksum.get(k, 0.0))
    achieved = per_launch[dom] / (kavg[dom] / 1e3) / 1e12
    peak = PEAK[args.precision]
    tile = (tuned.get(dom, {}).get("tile")
            or run.ctx.variants(dom_op[dom], prec)[run.ctx.get_variant(dom_op[dom], prec)])
    rec = measured_record(dom, tile, args.precision, cfg.name, args.q_batch)
    roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": round(peak, 1),
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
            "traffic": rec["traffic_bytes"] if rec else None,
            "kernel": dom, "tile": tile, "flop_per_launch": per_launch[dom],
            "avg_launch_ms": round(kavg[dom], 3)}
    if rec:
        # the executed MFMA work (Hermitian savings and tile padding included) from the counters
        ex = rec["mfma_bf16_flop_executed"] / (kavg[dom] / 1e3) / 1e12
        roof["executed_bf16_tflops"] = round(ex, 1)
        roof["executed_bf16_frac"] = round(ex / PEAK_BF16, 4)
    if args.precision == "bf16x3":
        roof["peak_basis"] = ("bf16 dense 2516.6 TFLOP/s / 3 products per split product; achieved "
                              "counts the dense complex flop model, executed_* the MFMA work done")
    kernels = {k: {"ms_per_step": round(ksum[k], 3), "launches_per_step": len(kern[k]) // kern_steps}
               for k in kern}
    kernels["polarization"]["tflops"] = round(fp / (ksum["polarization"] / 1e3) / 1e12, 2)
    kernels["self_energy"]["tflops"] = round(fs / (ksum["self_energy"] / 1e3) / 1e12, 2)

    # the FP64 GPU path on the same inputs (a q subset, same shapes)
    fp64_ref = None
    if args.fp64_ref_q > 0 and args.precision != "fp64":
        nq = args.fp64_ref_q
        ref = amd.GWRun(cfg.nk, prob.kmq, prob.nb, prob.ni, prob.tau, cfg.beta, cfg.niw_f,
                        cfg.niw_b, cfg.scale, prob.eps, prob.v, prob.n_target,
                        precision=amd.FP64, q_batch=nq)
        M64 = torch.empty(int(ref.mpre[nq]), dtype=torch.complex128, device="cuda")
        ref.ctx.synth_M(cfg.seed, 0, nq, 1, amd.C128, M64)
        ref.green0(0.0)
        t64 = EventTimer()
        ref.timer = t64
        ref.sig_tau.zero_()
        ref.sig_x.zero_()
        ref.q_block(amd.ResidentM(M64, ref.mpre), 0, nq)
        k64 = t64.summary()
        fp1 = fp * nq / cfg.nk
        fs1 = fs * nq / cfg.nk
        tp, ts = k64["polarization"][0] / 1e3, k64["self_energy"][0] / 1e3
        fp64_ref = {"q_points": nq, "polarization_tflops": round(fp1 / tp / 1e12, 2),
                    "self_energy_tflops": round(fs1 / ts / 1e12, 2),
                    "p_plus_sigma_tflops": round((fp1 + fs1) / (tp + ts) / 1e12, 2),
                    "p_plus_sigma_s_extrapolated": round((tp + ts) * cfg.nk / nq, 2),
                    "peak": PEAK["fp64"]}
        del M64, ref
        torch.cuda.empty_cache()

    cpu = None if args.no_cpu_baseline else cpu_baseline(cfg, prob)

    line = {
        "metric": "P+Sigma effective TFLOP/s and s per scGW iteration, split-FP32 vs FP64 GPU",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 2),
        "s_per_iteration": round(ms_step / 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f16x3": "f16x3 (split fp32 on f16 MFMA, scaled, fp32 accumulate) + f64",
                  "bf16x3": "bf16x3 (split fp32 on bf16 MFMA, fp32 accumulate) + f64",
                  "fp32": "f32 MFMA + f64", "fp64": "f64"}[args.precision],
        "data": "synthetic (seeded Philox matrix elements, model bands, diagonal Coulomb kernel)",
        "config": {"workload": f"{cfg.name}: one G0W0 + Dyson pass, all 64 q",
                   "nk": cfg.nk, "nb": int(prob.nb.max()), "ni": int(prob.ni.max()),
                   "ntau": int(prob.tau.size), "niw_f": cfg.niw_f, "niw_b": cfg.niw_b,
                   "beta": cfg.beta, "precision": args.precision, "q_batch": args.q_batch,
                   "hip_graph": bool(args.graph), "tau_mirror": bool(args.tau_mirror),
                   "flops_p": fp, "flops_sigma": fs},
        "roofline": roof,
        "kernels": kernels,
        "fp64_gpu_reference": fp64_ref,
        "cpu_baseline": cpu,
        "m_generation_s": round(t_gen, 3),
        "autotune": tuned,
        "check": {"flags": flags, "N": N, "n_target": prob.n_target, "gap_Ha": gap},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
