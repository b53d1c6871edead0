"""ctypes binding of libmatsgw.so: argument marshalling only.

Every method of :class:`Context` maps one-to-one onto an ``msgw_*`` entry point
of ``include/matsgw.h`` (same name without the prefix).  Device buffers are
torch tensors on the GPU (or raw integer addresses); the stream defaults to
torch's current stream.  Nothing here computes any part of the method: if the
shared library is missing the import fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmatsgw.so")

OK, EINVAL, ESHAPE, EHIP, ENOMEM, ENOCONV, ENOTSUP = 0, -1, -2, -3, -4, -5, -6
FP64, FP32, BF16X3, F16X3 = 0, 1, 2, 3
C128, C64 = 0, 1
FERMION, BOSON = 0, 1
SIGMA_DIAG, SIGMA_FULL = 0, 1
MU_FIXED, MU_SEARCH = 0, 1
FLAG_NAN, FLAG_NOBRACKET, FLAG_NOCONV, FLAG_SINGULAR = 1, 2, 4, 8
MAX_NI = 1024

EXPORTS = [
    "msgw_create", "msgw_destroy", "msgw_last_error", "msgw_set_problem",
    "msgw_workspace_size", "msgw_set_workspace", "msgw_m_layout", "msgw_green0",
    "msgw_polarization", "msgw_tau_to_iw", "msgw_iw_to_tau", "msgw_screen",
    "msgw_screened_tau", "msgw_self_energy", "msgw_sigma_x", "msgw_dyson", "msgw_gap",
    "msgw_synth_M", "msgw_variant_count", "msgw_variant_name", "msgw_set_variant", "msgw_get_variant",
    "msgw_set_k_range", "msgw_continue_pade", "msgw_gap_of", "msgw_set_tau_mirror",
    "msgw_continue_cpe", "msgw_dyson_noalloc", "msgw_set_kernel_events", "msgw_dyson_matrix",
    "msgw_tau_solver_work_size", "msgw_wt_tau_system", "msgw_dyson_tau",
    "msgw_set_symmetry", "msgw_ibz", "msgw_sigma_star", "msgw_synth_M_cubic",
]
OP_POLARIZATION, OP_SELF_ENERGY = 0, 1
TS_WTILDE, TS_DYSON = 0, 1


class MsgwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"matsgw error {code}: {msg}")
        self.code = code


class _Problem(ctypes.Structure):
    _fields_ = [
        ("nk", ctypes.c_int), ("kmq", ctypes.POINTER(ctypes.c_int)),
        ("nb", ctypes.POINTER(ctypes.c_int)), ("ni", ctypes.POINTER(ctypes.c_int)),
        ("ntau", ctypes.c_int), ("tau", ctypes.POINTER(ctypes.c_double)),
        ("beta", ctypes.c_double), ("niw_f", ctypes.c_int), ("niw_b", ctypes.c_int),
        ("scale", ctypes.c_double), ("sigma_mode", ctypes.c_int),
    ]


_lib = None


def load_library():
    """Load libmatsgw.so and declare the signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1602_02313_amd.build` (or __graft_entry__.build())")
    # torch bundles its own HIP runtime under the same soname (libamdhip64.so.7); load it first so
    # the library and torch's allocator and streams share one runtime in the process.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, I, L, D, U64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
    sig = {
        "msgw_create": [ctypes.POINTER(P), I],
        "msgw_destroy": [P],
        "msgw_set_problem": [P, ctypes.POINTER(_Problem)],
        "msgw_workspace_size": [P, I, ctypes.POINTER(ctypes.c_size_t)],
        "msgw_set_workspace": [P, P, ctypes.c_size_t],
        "msgw_m_layout": [P, I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
        "msgw_green0": [P, P, P, D, P],
        "msgw_polarization": [P, P, I, I, P, I, P, I, P],
        "msgw_tau_to_iw": [P, P, I, L, L, P, I, P, P],
        "msgw_iw_to_tau": [P, P, I, L, L, I, P, P, P, P],
        "msgw_screen": [P, P, I, I, P, P, P, P, P, P],
        "msgw_screened_tau": [P, P, I, I, P, P, P, P],
        "msgw_self_energy": [P, P, I, I, P, I, P, P, I, P],
        "msgw_sigma_x": [P, P, I, I, P, I, P, P, P],
        "msgw_dyson": [P, P, P, P, P, D, I, P, P, P, P, P],
        "msgw_dyson_noalloc": [P, P, P, P, P, D, I, P, P, P, P, P],
        "msgw_set_kernel_events": [P, I, P, P],
        "msgw_dyson_matrix": [P, P, P, P, P, D, I, P, P, P, P, P],
        "msgw_gap": [P, P, P, P, P, P, I, P],
        "msgw_synth_M": [P, P, U64, I, I, I, I, P],
        "msgw_tau_solver_work_size": [P, I, I, I, ctypes.POINTER(ctypes.c_size_t)],
        "msgw_wt_tau_system": [P, P, I, I, P, P, P, P, P, ctypes.c_size_t],
        "msgw_dyson_tau": [P, P, I, I, P, P, P, P, P, P, P, ctypes.c_size_t],
        "msgw_set_symmetry": [P, I, ctypes.POINTER(ctypes.c_int)],
        "msgw_ibz": [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
        "msgw_sigma_star": [P, P, I, P, P, P, P],
        "msgw_synth_M_cubic": [P, P, U64, I, I, I, P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.msgw_last_error.argtypes = [P]
    lib.msgw_last_error.restype = ctypes.c_char_p
    lib.msgw_variant_count.argtypes = [I, I]
    lib.msgw_variant_count.restype = ctypes.c_int
    lib.msgw_variant_name.argtypes = [I, I, I]
    lib.msgw_variant_name.restype = ctypes.c_char_p
    lib.msgw_set_variant.argtypes = [P, I, I, I]
    lib.msgw_set_variant.restype = ctypes.c_int
    lib.msgw_get_variant.argtypes = [P, I, I, ctypes.POINTER(ctypes.c_int)]
    lib.msgw_get_variant.restype = ctypes.c_int
    lib.msgw_set_k_range.argtypes = [P, I, I, I]
    lib.msgw_set_k_range.restype = ctypes.c_int
    lib.msgw_continue_pade.argtypes = [P, P, I, ctypes.c_double, P, P, P, P, I, P, P, P, P]
    lib.msgw_continue_pade.restype = ctypes.c_int
    lib.msgw_gap_of.argtypes = [P, P, P, I, P]
    lib.msgw_gap_of.restype = ctypes.c_int
    lib.msgw_continue_cpe.argtypes = [P, P, I, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      P, P, P, P, I, P, P, P, P, P]
    lib.msgw_continue_cpe.restype = ctypes.c_int
    lib.msgw_set_tau_mirror.argtypes = [P, I]
    lib.msgw_set_tau_mirror.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(x):
    """Device address of a tensor (or an int address, or None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        if not x.is_cuda:
            raise ValueError("device buffer expected (got a CPU tensor)")
        if not x.is_contiguous():
            raise ValueError("contiguous buffer expected")
        return x.data_ptr()
    raise TypeError(f"cannot pass {type(x)} as a device pointer")


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


class Context:
    """One msgw_ctx bound to a HIP device."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        self._c = ctypes.c_void_p()
        rc = self.lib.msgw_create(ctypes.byref(self._c), device)
        if rc != OK:
            raise MsgwError(rc, f"msgw_create(device={device}) failed")
        self.device = device
        self._keep = []

    def close(self):
        if self._c:
            self.lib.msgw_destroy(self._c)
            self._c = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != OK:
            msg = self.lib.msgw_last_error(self._c)
            raise MsgwError(rc, msg.decode() if msg else "")
        return rc

    # ---- context ----
    def set_problem(self, nk, kmq, nb, ni, tau, beta, niw_f, niw_b, scale,
                    sigma_mode=SIGMA_DIAG):
        kmq = np.ascontiguousarray(np.asarray(kmq, dtype=np.int32).reshape(-1))
        nb = np.ascontiguousarray(np.asarray(nb, dtype=np.int32))
        ni = np.ascontiguousarray(np.asarray(ni, dtype=np.int32))
        tau = np.ascontiguousarray(np.asarray(tau, dtype=np.float64))
        p = _Problem(int(nk), kmq.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                     nb.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                     ni.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), int(tau.size),
                     tau.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(beta),
                     int(niw_f), int(niw_b), float(scale), int(sigma_mode))
        self._check(self.lib.msgw_set_problem(self._c, ctypes.byref(p)))
        self._nk = int(nk)

    def workspace_size(self, nq_max=1):
        b = ctypes.c_size_t()
        self._check(self.lib.msgw_workspace_size(self._c, int(nq_max), ctypes.byref(b)))
        return int(b.value)

    def set_workspace(self, buf, nbytes=None):
        if nbytes is None:
            nbytes = buf.numel() * buf.element_size()
        self._check(self.lib.msgw_set_workspace(self._c, _ptr(buf), int(nbytes)))
        self._keep = [buf]

    def m_layout(self, q, nk):
        off = np.zeros(nk, dtype=np.int64)
        qs = ctypes.c_int64()
        self._check(self.lib.msgw_m_layout(self._c, int(q),
                                           off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                           ctypes.byref(qs)))
        return off, int(qs.value)

    # ---- hot path ----
    def green0(self, eps, mu, G_tau, stream=None):
        self._check(self.lib.msgw_green0(self._c, _stream(stream), _ptr(eps), float(mu), _ptr(G_tau)))

    def polarization(self, q0, nq, M, m_dtype, G_tau, precision, P_tau, stream=None):
        self._check(self.lib.msgw_polarization(self._c, _stream(stream), q0, nq, _ptr(M), m_dtype,
                                               _ptr(G_tau), precision, _ptr(P_tau)))

    def tau_to_iw(self, stat, nblk, length, f_tau, f_is_complex, e_ref, f_iw, stream=None):
        self._check(self.lib.msgw_tau_to_iw(self._c, _stream(stream), stat, int(nblk), int(length),
                                            _ptr(f_tau), int(f_is_complex), _ptr(e_ref), _ptr(f_iw)))

    def iw_to_tau(self, stat, nblk, length, mat_n, f_iw, add_tau, e_ref, f_tau, stream=None):
        self._check(self.lib.msgw_iw_to_tau(self._c, _stream(stream), stat, int(nblk), int(length),
                                            int(mat_n), _ptr(f_iw), _ptr(add_tau), _ptr(e_ref),
                                            _ptr(f_tau)))

    def screen(self, q0, nq, P_iw, v, Wt_iw, R_iw, info, flags=None, stream=None):
        self._check(self.lib.msgw_screen(self._c, _stream(stream), q0, nq, _ptr(P_iw), _ptr(v),
                                         _ptr(Wt_iw), _ptr(R_iw), _ptr(info), _ptr(flags)))

    def screened_tau(self, q0, nq, R_iw, P_tau, v, Wt_tau, stream=None):
        self._check(self.lib.msgw_screened_tau(self._c, _stream(stream), q0, nq, _ptr(R_iw),
                                               _ptr(P_tau), _ptr(v), _ptr(Wt_tau)))

    def self_energy(self, q0, nq, M, m_dtype, G_tau, Wt_tau, precision, Sigma_tau, stream=None):
        self._check(self.lib.msgw_self_energy(self._c, _stream(stream), q0, nq, _ptr(M), m_dtype,
                                              _ptr(G_tau), _ptr(Wt_tau), precision, _ptr(Sigma_tau)))

    def sigma_x(self, q0, nq, M, m_dtype, G_tau, v, Sigma_x, stream=None):
        self._check(self.lib.msgw_sigma_x(self._c, _stream(stream), q0, nq, _ptr(M), m_dtype,
                                          _ptr(G_tau), _ptr(v), _ptr(Sigma_x)))

    def dyson(self, eps, sigma_static, Sigma_c_iw, n_target, mu_mode, mu, G_iw, G_tau, n_out,
              flags, stream=None):
        self._check(self.lib.msgw_dyson(self._c, _stream(stream), _ptr(eps), _ptr(sigma_static),
                                        _ptr(Sigma_c_iw), float(n_target), int(mu_mode), _ptr(mu),
                                        _ptr(G_iw), _ptr(G_tau), _ptr(n_out), _ptr(flags)))

    def dyson_matrix(self, eps, sigma_static, Sigma_c_iw, n_target, mu_mode, mu, G_iw, G_tau, n_out,
                     flags, stream=None):
        self._check(self.lib.msgw_dyson_matrix(self._c, _stream(stream), _ptr(eps), _ptr(sigma_static),
                                               _ptr(Sigma_c_iw), float(n_target), int(mu_mode), _ptr(mu),
                                               _ptr(G_iw), _ptr(G_tau), _ptr(n_out), _ptr(flags)))

    def dyson_noalloc(self, eps, sigma_static, Sigma_c_iw, n_target, mu_mode, mu, G_iw, G_tau, n_out,
                      flags, stream=None):
        self._check(self.lib.msgw_dyson_noalloc(self._c, _stream(stream), _ptr(eps), _ptr(sigma_static),
                                                _ptr(Sigma_c_iw), float(n_target), int(mu_mode), _ptr(mu),
                                                _ptr(G_iw), _ptr(G_tau), _ptr(n_out), _ptr(flags)))

    def tau_solver_work_size(self, which, first, count):
        b = ctypes.c_size_t(0)
        self._check(self.lib.msgw_tau_solver_work_size(self._c, int(which), int(first), int(count),
                                                       ctypes.byref(b)))
        return b.value

    def wt_tau_system(self, q0, nq, P_tau, v, Wt_tau, info, work, work_bytes, stream=None):
        self._check(self.lib.msgw_wt_tau_system(self._c, _stream(stream), int(q0), int(nq), _ptr(P_tau), _ptr(v),
                                                _ptr(Wt_tau), _ptr(info), _ptr(work), int(work_bytes)))

    def dyson_tau(self, k0, nkc, eps, sigma_static, mu, Sigma_c_tau, G_tau, info, work, work_bytes,
                  stream=None):
        self._check(self.lib.msgw_dyson_tau(self._c, _stream(stream), int(k0), int(nkc), _ptr(eps),
                                            _ptr(sigma_static), _ptr(mu), _ptr(Sigma_c_tau), _ptr(G_tau),
                                            _ptr(info), _ptr(work), int(work_bytes)))

    def set_symmetry(self, rot_k):
        r = np.ascontiguousarray(rot_k, dtype=np.int32)
        self._check(self.lib.msgw_set_symmetry(self._c, int(r.shape[0]),
                                               r.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))

    def ibz(self):
        """(irreducible q list, star sizes)."""
        n = ctypes.c_int(0)
        nk = self._nk
        q = (ctypes.c_int * nk)()
        st = (ctypes.c_int * nk)()
        self._check(self.lib.msgw_ibz(self._c, ctypes.byref(n), q, st))
        return list(q[:n.value]), list(st[:n.value])

    def sigma_star(self, q_ibz, C_tau, C_x, Sigma_tau, Sigma_x, stream=None):
        self._check(self.lib.msgw_sigma_star(self._c, _stream(stream), int(q_ibz), _ptr(C_tau), _ptr(C_x),
                                             _ptr(Sigma_tau), _ptr(Sigma_x)))

    def synth_M_cubic(self, seed, q0, nq, m_dtype, M, stream=None):
        self._check(self.lib.msgw_synth_M_cubic(self._c, _stream(stream), int(seed), int(q0), int(nq),
                                                int(m_dtype), _ptr(M)))

    def gap(self, eps, sigma_static, Sigma_c_iw, mu, n_index, gap, stream=None):
        self._check(self.lib.msgw_gap(self._c, _stream(stream), _ptr(eps), _ptr(sigma_static),
                                      _ptr(Sigma_c_iw), _ptr(mu), int(n_index), _ptr(gap)))

    def variants(self, op, precision):
        """Names of the compiled tile-shape variants of an MFMA op."""
        n = self.lib.msgw_variant_count(int(op), int(precision))
        if n < 0:
            raise MsgwError(n, "bad op or precision")
        return [self.lib.msgw_variant_name(int(op), int(precision), v).decode() for v in range(n)]

    def set_variant(self, op, precision, variant):
        self._check(self.lib.msgw_set_variant(self._c, int(op), int(precision), int(variant)))

    def get_variant(self, op, precision):
        out = ctypes.c_int(-1)
        rc = self.lib.msgw_get_variant(self._c, int(op), int(precision), ctypes.byref(out))
        if rc != 0:
            raise MsgwError(rc, "bad op or precision")
        return out.value

    def continue_pade(self, n_pade, eta, eps, sigma_static, Sigma_c_iw, mu, omega, A, E_qp, flags,
                      stream=None):
        n_omega = 0 if omega is None else int(omega.numel())
        self._check(self.lib.msgw_continue_pade(self._c, _stream(stream), int(n_pade), float(eta), _ptr(eps),
                                                _ptr(sigma_static), _ptr(Sigma_c_iw), _ptr(mu), n_omega,
                                                _ptr(omega), _ptr(A), _ptr(E_qp), _ptr(flags)))

    def set_tau_mirror(self, on=True):
        """Assert P(tau) = P(beta - tau) for the inputs (time-reversal symmetry); see matsgw.h."""
        self._check(self.lib.msgw_set_tau_mirror(self._c, int(bool(on))))

    def continue_cpe(self, n_real, w_min, w_max, ridge, eta, eps, sigma_static, Sigma_c_iw, mu, omega, A, E_qp,
                     coef, flags, stream=None):
        n_omega = 0 if omega is None else int(omega.numel())
        self._check(self.lib.msgw_continue_cpe(self._c, _stream(stream), int(n_real), float(w_min), float(w_max),
                                               float(ridge), float(eta), _ptr(eps), _ptr(sigma_static),
                                               _ptr(Sigma_c_iw), _ptr(mu), n_omega, _ptr(omega), _ptr(A),
                                               _ptr(E_qp), _ptr(coef), _ptr(flags)))

    def gap_of(self, E, n_index, gap, stream=None):
        self._check(self.lib.msgw_gap_of(self._c, _stream(stream), _ptr(E), int(n_index), _ptr(gap)))

    def set_k_range(self, k0=0, k1=0, reuse_prepared=False):
        """Harness only: restrict the pair-space contractions to k blocks [k0, k1) (k1 <= 0: all)."""
        self._check(self.lib.msgw_set_k_range(self._c, int(k0), int(k1), int(bool(reuse_prepared))))

    def set_kernel_events(self, op, start=None, stop=None):
        """Harness only: record the torch.cuda.Events start / stop around the contraction kernels of the
        following calls of op (None, None: stop).  The events must have been recorded once (torch
        creates them lazily)."""
        a = None if start is None else ctypes.c_void_p(start.cuda_event)
        b = None if stop is None else ctypes.c_void_p(stop.cuda_event)
        self._check(self.lib.msgw_set_kernel_events(self._c, int(op), a, b))

    def synth_M(self, seed, q0, nq, symmetric, m_dtype, M, stream=None):
        self._check(self.lib.msgw_synth_M(self._c, _stream(stream), int(seed), q0, nq,
                                          int(symmetric), m_dtype, _ptr(M)))
