"""Tile-shape autotuner for the MFMA contractions.

Each compiled variant (msgw_variant_name) of the polarization and self-energy kernels is
launched on the run's own shapes (the first q batch), timed with HIP events, and the fastest is
selected on the context (variants within 2% of the fastest count as ties, won by the lower index).  Results can be cached in a JSON file keyed by the problem shape.
"""
from __future__ import annotations

import json
import os

from . import _lib as L

TIE = 0.02  # relative time difference below which the earlier (default-order) variant is kept


def pick(times, tie=TIE):
    """Index of the lowest-index variant within `tie` (relative) of the fastest finite time."""
    fastest = min(times)
    if fastest == float("inf"):
        raise RuntimeError("no tile variant can run these shapes")
    return next(v for v, t in enumerate(times) if t <= fastest * (1.0 + tie))


def _key(run, op):
    return "|".join(str(x) for x in (op, run.precision, run.nk, int(run.nb.max()), int(run.ni.max()),
                                     run.ntau, run.q_batch))


def _launch(op, ctx, run, M, q0, nq, st):
    if op == L.OP_POLARIZATION:
        ctx.polarization(q0, nq, M, run.m_dtype, run.G_tau, run.precision, run.P_tau, stream=st)
    else:
        ctx.self_energy(q0, nq, M, run.m_dtype, run.G_tau, run.Wt_tau, run.precision, run.sig_tau,
                        stream=st)


def tune(run, M_source, reps=2, cache_path=None, log=None, ops=None, nq=None):
    """Pick the fastest variant of each MFMA op for `run`; returns {op: (index, name, ms list)}.

    The variants are timed on q = 0 .. nq - 1 (default: the run's q batch)."""
    import torch
    if run.precision not in (L.FP32, L.BF16X3, L.F16X3):
        return {}
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    out = {}
    q0, nq = 0, min(run.q_batch if nq is None else nq, run.q_batch, run.nk)
    M = M_source(run, q0, nq)
    ctx, st = run.ctx, run.stream
    # realistic W~(tau) and G for the timing launches
    run.green0(0.0)
    run.sig_tau.zero_()
    run.sig_x.zero_()
    run.q_block(M_source, q0, nq)
    for op in (ops if ops is not None else (L.OP_POLARIZATION, L.OP_SELF_ENERGY)):
        names = ctx.variants(op, run.precision)
        key = _key(run, op)
        if key in cache and cache[key] < len(names):
            best = cache[key]
            ctx.set_variant(op, run.precision, best)
            out[op] = (best, names[best], None)
            continue
        times = []
        for v in range(len(names)):
            ctx.set_variant(op, run.precision, v)
            ms = []
            try:
                _launch(op, ctx, run, M, q0, nq, st)
            except L.MsgwError as e:  # this tile cannot run these shapes
                times.append(float("inf"))
                if log:
                    log(f"[autotune] op={op} variant {v} ({names[v]}): unavailable ({e})")
                continue
            for r in range(reps):  # the launch above was the warm-up
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(st) if st is not None else a.record()
                _launch(op, ctx, run, M, q0, nq, st)
                b.record(st) if st is not None else b.record()
                torch.cuda.synchronize()
                ms.append(a.elapsed_time(b))
            times.append(min(ms))
            if log:
                log(f"[autotune] op={op} variant {v} ({names[v]}): {min(ms):.2f} ms")
        best = pick(times)
        ctx.set_variant(op, run.precision, best)
        out[op] = (best, names[best], times)
        cache[key] = best
    if cache_path:
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    run.sig_tau.zero_()
    run.sig_x.zero_()
    return out
