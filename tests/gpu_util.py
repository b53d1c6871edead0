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
