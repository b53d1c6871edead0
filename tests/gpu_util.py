"""Helpers shared by the GPU parity tests: build a GWRun from seeded inputs, compare arrays."""
import numpy as np

import gwinputs as gi


def rel(got, ref):
    """Frobenius-norm relative error ||got - ref|| / ||ref||."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    den = np.linalg.norm(ref.ravel())
    return float(np.linalg.norm((got - ref).ravel()) / (den if den > 0 else 1.0))


def make_run(cfg, precision=None, sigma_mode=None, q_batch=1):
    import paper_1602_02313_amd as amd
    prob = gi.make_problem(cfg)
    precision = amd.FP64 if precision is None else precision
    sigma_mode = amd.SIGMA_DIAG if sigma_mode is None else sigma_mode
    run = amd.GWRun(cfg.nk, prob.kmq, prob.nb, prob.ni, prob.tau, cfg.beta, cfg.niw_f, cfg.niw_b,
                    cfg.scale, prob.eps, prob.v, prob.n_target, precision=precision,
                    sigma_mode=sigma_mode, q_batch=q_batch)
    return prob, run


def host_M(cfg, m_dtype, symmetric=True):
    import paper_1602_02313_amd as amd
    g = gi.MGenerator(cfg, symmetric=symmetric)
    return g, amd.HostM(lambda q: g.q_packed(q), m_dtype)


def np_(t):
    return t.detach().cpu().numpy()


def slice_rel(got, ref, axis=-1):
    """Worst relative Frobenius error over the slices along `axis` (e.g. per tau point); slices
    whose reference is zero are measured against the largest slice norm."""
    got = np.moveaxis(np.asarray(got), axis, 0)
    ref = np.moveaxis(np.asarray(ref), axis, 0)
    dn = np.array([np.linalg.norm((g - r).ravel()) for g, r in zip(got, ref)])
    rn = np.array([np.linalg.norm(r.ravel()) for r in ref])
    floor = rn.max() if rn.size and rn.max() > 0 else 1.0
    return float(np.max(dn / np.where(rn > 0, rn, floor)))


def max_rel(got, ref):
    """max |got - ref| / max |ref| (the absolute maximum error on the reference's scale)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    den = np.abs(ref).max() if ref.size else 1.0
    return float(np.abs(got - ref).max() / (den if den > 0 else 1.0))


SLICE = 10.0  # worst tau slice and max-abs error are bounded by SLICE x the Frobenius gate


def check(name, got, ref, gate, tau_axis, slices=True):
    """Frobenius, worst-tau-slice and max-abs errors against the gate; returns the Frobenius error.

    slices=False bounds only the max-abs error beside the Frobenius norm: for W~(tau) the truncated
    Matsubara sum spreads an absolute error evenly over tau while W~ itself decays by orders of
    magnitude towards beta/2, so a slice's error relative to that slice measures the transform's
    conditioning, not the contraction (the worst slice is still printed)."""
    e, es, em = rel(got, ref), slice_rel(got, ref, tau_axis), max_rel(got, ref)
    print(f"{name}: rel {e:.2e}, worst tau slice {es:.2e}, max-abs {em:.2e}")
    assert e < gate, (name, e)
    assert em < SLICE * gate, (name, em)
    if slices:
        assert es < SLICE * gate, (name, es)
    return e
