"""Thin ctypes binding of the C ABI in include/qtx_rgf.h.

Argument marshalling only: every step of the solve runs in the HIP library
libqtx_rgf.so.  Device memory is handled by the caller (PyTorch complex128
tensors on the GPU); this module passes their data pointers.  Loading fails
loudly if the library has not been built.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# QTX_RGF_LIB selects another build of the library (e.g. a tuning variant)
LIB_PATH = os.environ.get("QTX_RGF_LIB") or os.path.join(_HERE, "libqtx_rgf.so")

QTX_OK = 0
QTX_ERR_INVALID_ARG = 1
QTX_ERR_SINGULAR = 2
QTX_ERR_NOT_FINITE = 3
QTX_ERR_NOMEM = 4
QTX_ERR_HIP = 5
QTX_ERR_BUSY = 6
QTX_ERR_PROBLEM = 7

QTX_KIND_G = 0
QTX_KIND_W = 1
QTX_FP64 = 0
QTX_MIXED = 1
QTX_FLAG_PROFILE = 1
QTX_NOALLOC_SCRATCH_BYTES = 64 << 20

KERNEL_CLASSES = {"zgemm": 0, "cgemm": 1, "inverse": 2, "elementwise": 3}


class BtIn(ctypes.Structure):
    _fields_ = [("diag", ctypes.c_void_p), ("upper", ctypes.c_void_p),
                ("lower", ctypes.c_void_p)]


class BtOut(ctypes.Structure):
    _fields_ = [("diag", ctypes.c_void_p), ("upper", ctypes.c_void_p),
                ("lower", ctypes.c_void_p)]


class Problem(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("n_blocks", ctypes.c_int32), ("block_size", ctypes.c_int32),
        ("n_energies", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("energies", ctypes.POINTER(ctypes.c_double)),
        ("H", BtIn), ("S", BtIn), ("sigma_r", BtIn), ("sigma_l", BtIn),
        ("sigma_g", BtIn),
        ("V", BtIn), ("P_r", BtIn), ("P_l", BtIn), ("P_g", BtIn),
        ("XR", BtOut), ("XL", BtOut), ("XG", BtOut),
        ("WR_diag", ctypes.c_void_p),
        ("status", ctypes.c_int32), ("fail_energy", ctypes.c_int32),
        ("fail_block", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class Nested(ctypes.Structure):
    _fields_ = [("n_partitions", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("reduced", BtOut), ("reduced_l", BtOut), ("reduced_g", BtOut)]


class Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("fail_energy", ctypes.c_int32), ("fail_block", ctypes.c_int32),
                ("n_energies", ctypes.c_int32), ("queue_s", ctypes.c_double),
                ("latency_s", ctypes.c_double)]


_lib = None


class QtxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


def lib():
    """Load libqtx_rgf.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqtx_rgf.so is not built (%s); run "
                          "python -m paper_2508_19138_amd.build" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    c_ctx = ctypes.c_void_p
    L.qtx_rgf_create.argtypes = [ctypes.POINTER(c_ctx), ctypes.c_int,
                                 ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint32]
    L.qtx_rgf_create.restype = ctypes.c_int
    L.qtx_rgf_solve_batch.argtypes = [c_ctx, ctypes.POINTER(Problem), ctypes.c_int32]
    L.qtx_rgf_solve_batch.restype = ctypes.c_int
    L.qtx_rgf_destroy.argtypes = [c_ctx]
    L.qtx_rgf_destroy.restype = ctypes.c_int
    L.qtx_rgf_status_string.argtypes = [ctypes.c_int]
    L.qtx_rgf_status_string.restype = ctypes.c_char_p
    L.qtx_rgf_last_error.argtypes = [c_ctx]
    L.qtx_rgf_last_error.restype = ctypes.c_char_p
    L.qtx_rgf_flops_per_energy.argtypes = [ctypes.c_int32] * 6
    L.qtx_rgf_flops_per_energy.restype = ctypes.c_double
    L.qtx_rgf_kernel_stats.argtypes = [c_ctx, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]
    L.qtx_rgf_kernel_stats.restype = ctypes.c_int
    L.qtx_rgf_reset_stats.argtypes = [c_ctx]
    L.qtx_rgf_reset_stats.restype = ctypes.c_int
    gemm_args = [c_ctx, ctypes.c_char, ctypes.c_char, ctypes.c_int32,
                 ctypes.c_int32, ctypes.c_int32]
    ptr_ld_s = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64]
    L.qtx_rgf_zgemm.argtypes = (gemm_args + [ctypes.c_double, ctypes.c_double]
                                + ptr_ld_s + ptr_ld_s
                                + [ctypes.c_double, ctypes.c_double]
                                + ptr_ld_s + ptr_ld_s + [ctypes.c_int32])
    L.qtx_rgf_zgemm.restype = ctypes.c_int
    L.qtx_rgf_cgemm.argtypes = L.qtx_rgf_zgemm.argtypes
    L.qtx_rgf_cgemm.restype = ctypes.c_int
    L.qtx_rgf_zinv.argtypes = [c_ctx, ctypes.c_int32, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
    L.qtx_rgf_zinv.restype = ctypes.c_int
    L.qtx_rgf_zinv_noalloc.argtypes = L.qtx_rgf_zinv.argtypes
    L.qtx_rgf_solve_nested.argtypes = [c_ctx, ctypes.POINTER(Problem), ctypes.POINTER(Nested)]
    L.qtx_rgf_solve_nested.restype = ctypes.c_int
    L.qtx_rgf_zinv_noalloc.restype = ctypes.c_int
    L.qtx_rgf_obc_fixed_point.argtypes = [
        c_ctx, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
        ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_int32]
    L.qtx_rgf_obc_fixed_point.restype = ctypes.c_int
    L.qtx_rgf_obc_sancho_rubio.argtypes = L.qtx_rgf_obc_fixed_point.argtypes
    L.qtx_rgf_obc_sancho_rubio.restype = ctypes.c_int
    L.qtx_rgf_obc_lesser_greater.argtypes = [
        c_ctx, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.qtx_rgf_obc_lesser_greater.restype = ctypes.c_int
    L.qtx_rgf_observables.argtypes = [
        c_ctx, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p]
    L.qtx_rgf_observables.restype = ctypes.c_int
    L.qtx_rgf_energy_convolution.argtypes = [
        c_ctx, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
        ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
        ctypes.c_double, ctypes.c_double]
    L.qtx_rgf_energy_convolution.restype = ctypes.c_int
    lyap = [c_ctx, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
    L.qtx_rgf_obc_lyapunov_fixed_point.argtypes = lyap
    L.qtx_rgf_obc_lyapunov_fixed_point.restype = ctypes.c_int
    L.qtx_rgf_obc_lyapunov_doubling.argtypes = lyap
    L.qtx_rgf_obc_lyapunov_doubling.restype = ctypes.c_int
    L.qtx_rgf_submit.argtypes = [c_ctx, ctypes.POINTER(Problem),
                                 ctypes.POINTER(ctypes.c_uint64)]
    L.qtx_rgf_submit.restype = ctypes.c_int
    L.qtx_rgf_poll.argtypes = [c_ctx, ctypes.POINTER(Completion), ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
    L.qtx_rgf_poll.restype = ctypes.c_int
    _lib = L
    return L


def exported_symbols():
    return ["qtx_rgf_create", "qtx_rgf_solve_batch", "qtx_rgf_destroy",
            "qtx_rgf_status_string", "qtx_rgf_last_error",
            "qtx_rgf_flops_per_energy", "qtx_rgf_kernel_stats",
            "qtx_rgf_reset_stats", "qtx_rgf_zgemm", "qtx_rgf_cgemm",
            "qtx_rgf_zinv", "qtx_rgf_zinv_noalloc", "qtx_rgf_submit", "qtx_rgf_poll",
            "qtx_rgf_solve_nested",
            "qtx_rgf_obc_fixed_point", "qtx_rgf_obc_sancho_rubio",
            "qtx_rgf_obc_lesser_greater", "qtx_rgf_observables",
            "qtx_rgf_obc_lyapunov_fixed_point", "qtx_rgf_obc_lyapunov_doubling",
            "qtx_rgf_energy_convolution"]


def status_string(st):
    return lib().qtx_rgf_status_string(st).decode()


def flops_per_energy(kind, n, b, n_rhs=2, bt_rhs=False, want_wr=False):
    return lib().qtx_rgf_flops_per_energy(kind, n, b, n_rhs, int(bt_rhs), int(want_wr))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _bt_in(d=None, u=None, l=None):
    return BtIn(_ptr(d), _ptr(u), _ptr(l))


def _bt_out(d=None, u=None, l=None):
    return BtOut(_ptr(d), _ptr(u), _ptr(l))


class Context:
    """qtx_rgf_create / qtx_rgf_destroy around one device."""

    def __init__(self, device=0, budget_bytes=0, stream=None, profile=False):
        L = lib()
        self._h = ctypes.c_void_p()
        flags = QTX_FLAG_PROFILE if profile else 0
        st = L.qtx_rgf_create(ctypes.byref(self._h), device, budget_bytes,
                              stream, flags)
        if st != QTX_OK:
            raise QtxError(st, "qtx_rgf_create: " + status_string(st))

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().qtx_rgf_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def last_error(self):
        return lib().qtx_rgf_last_error(self._h).decode()

    def _check(self, st, what):
        if st not in (QTX_OK, QTX_ERR_PROBLEM):
            raise QtxError(st, "%s: %s (%s)" % (what, status_string(st), self.last_error()))
        return st

    def solve_batch(self, problems):
        """problems: list of Problem structures (see make_g_problem etc.).
        Returns the call status; per-problem status is in each structure."""
        arr = (Problem * len(problems))(*problems)
        st = lib().qtx_rgf_solve_batch(self._h, arr, len(problems))
        for i, p in enumerate(problems):
            p.status = arr[i].status
            p.fail_energy = arr[i].fail_energy
            p.fail_block = arr[i].fail_block
        return self._check(st, "qtx_rgf_solve_batch")

    def solve_nested(self, problem, n_partitions, reduced=None, reduced_l=None,
                     reduced_g=None):
        """One problem by the partitioned scheme.  reduced / reduced_l /
        reduced_g: optional (diag, upper, lower) device tensors receiving the
        reduced system and right-hand sides (lower unused for the latter)."""
        o = Nested(n_partitions, 0,
                   _bt_out(*(reduced or (None, None, None))),
                   _bt_out(*(reduced_l or (None, None, None))),
                   _bt_out(*(reduced_g or (None, None, None))))
        st = lib().qtx_rgf_solve_nested(self._h, ctypes.byref(problem), ctypes.byref(o))
        return self._check(st, "qtx_rgf_solve_nested")

    def submit(self, problem):
        """Queue one problem on the request loop; returns its ticket.  The
        caller keeps the problem's device buffers alive until its completion
        has been polled."""
        t = ctypes.c_uint64()
        st = lib().qtx_rgf_submit(self._h, ctypes.byref(problem), ctypes.byref(t))
        self._check(st, "qtx_rgf_submit")
        return t.value

    def poll(self, cap=64, wait_ms=0):
        """Return (completions, n_pending); each completion is a dict."""
        out = (Completion * max(cap, 1))()
        n, pend = ctypes.c_int32(), ctypes.c_int32()
        st = lib().qtx_rgf_poll(self._h, out, cap, ctypes.byref(n),
                                ctypes.byref(pend), wait_ms)
        self._check(st, "qtx_rgf_poll")
        res = [{"ticket": out[i].ticket, "status": out[i].status,
                "fail_energy": out[i].fail_energy, "fail_block": out[i].fail_block,
                "n_energies": out[i].n_energies, "queue_s": out[i].queue_s,
                "latency_s": out[i].latency_s} for i in range(n.value)]
        return res, pend.value

    def kernel_stats(self, cls):
        n = ctypes.c_int64()
        ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        st = lib().qtx_rgf_kernel_stats(self._h, KERNEL_CLASSES.get(cls, cls),
                                        ctypes.byref(n), ctypes.byref(ms),
                                        ctypes.byref(fl), ctypes.byref(by))
        self._check(st, "qtx_rgf_kernel_stats")
        return {"launches": n.value, "ms": ms.value, "flops": fl.value,
                "bytes": by.value}

    def reset_stats(self):
        lib().qtx_rgf_reset_stats(self._h)

    def zgemm(self, opa, opb, m, n, k, alpha, A, lda, sA, B, ldb, sB, beta,
              C, ldc, sC, D, ldd, sD, batch, fp32=False):
        fn = lib().qtx_rgf_cgemm if fp32 else lib().qtx_rgf_zgemm
        st = fn(self._h, opa.encode(), opb.encode(), m, n, k,
                alpha.real, alpha.imag, _ptr(A), lda, sA,
                _ptr(B), ldb, sB, beta.real, beta.imag,
                _ptr(C), ldc, sC, _ptr(D), ldd, sD, batch)
        return self._check(st, "qtx_rgf_cgemm" if fp32 else "qtx_rgf_zgemm")

    def zinv(self, b, A, X, info, batch):
        st = lib().qtx_rgf_zinv(self._h, b, _ptr(A), _ptr(X), _ptr(info), batch)
        return self._check(st, "qtx_rgf_zinv")

    def zinv_noalloc(self, b, A, X, info, batch):
        """Asynchronous on the context's stream: synchronise before reading X."""
        st = lib().qtx_rgf_zinv_noalloc(self._h, b, _ptr(A), _ptr(X), _ptr(info), batch)
        return self._check(st, "qtx_rgf_zinv_noalloc")

    def obc_fixed_point(self, b, batch, m, s_m, n, s_n, n_prime, s_np, x, sigma,
                        update, info, n_iter):
        """n_iter iterations of x <- (m - n x n')^{-1}; see the C header.
        Strides in complex elements between energies (0 = shared block)."""
        st = lib().qtx_rgf_obc_fixed_point(self._h, b, batch, _ptr(m), s_m, _ptr(n), s_n,
                                           _ptr(n_prime), s_np, _ptr(x), _ptr(sigma),
                                           _ptr(update), _ptr(info), n_iter)
        return self._check(st, "qtx_rgf_obc_fixed_point")

    def obc_sancho_rubio(self, b, batch, m, s_m, n, s_n, n_prime, s_np, x, sigma,
                         coupling, info, n_steps):
        """n_steps decimation steps, then x = m_surf^{-1}; see the C header."""
        st = lib().qtx_rgf_obc_sancho_rubio(self._h, b, batch, _ptr(m), s_m, _ptr(n), s_n,
                                            _ptr(n_prime), s_np, _ptr(x), _ptr(sigma),
                                            _ptr(coupling), _ptr(info), n_steps)
        return self._check(st, "qtx_rgf_obc_sancho_rubio")

    def obc_lesser_greater(self, b, batch, sigma_r, s_sr, f, one_minus_f, sigma_l, sigma_g):
        """Sigma^< = i f Gamma, Sigma^> = -i (1-f) Gamma; f, one_minus_f are host
        float64 numpy arrays of length batch (kept alive by the caller)."""
        fp = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
        gp = None if one_minus_f is None else np.ascontiguousarray(one_minus_f, dtype=np.float64)
        for a in (fp, gp):
            if a is not None and a.size < batch:
                raise ValueError("occupation arrays need one value per energy")
        dp = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        st = lib().qtx_rgf_obc_lesser_greater(self._h, b, batch, _ptr(sigma_r), s_sr, dp(fp),
                                              dp(gp), _ptr(sigma_l), _ptr(sigma_g))
        return self._check(st, "qtx_rgf_obc_lesser_greater")

    def observables(self, n, b, batch, XL_diag, XG_diag, XL_lower, H_upper, dos, density,
                    current):
        """Density of states, density and current per block; see the C header."""
        st = lib().qtx_rgf_observables(self._h, n, b, batch, _ptr(XL_diag), _ptr(XG_diag),
                                       _ptr(XL_lower), _ptr(H_upper), _ptr(dos),
                                       _ptr(density), _ptr(current))
        return self._check(st, "qtx_rgf_observables")

    def energy_convolution(self, n_elem, X1, n1, X2, n2, B, n_out, shift=0, scale=1.0,
                           reverse1=False):
        """B[k][i] = scale * sum_k' X1'[k + shift - k'][i] X2[k'][i]; see the C header."""
        s = complex(scale)
        st = lib().qtx_rgf_energy_convolution(self._h, n_elem, _ptr(X1), n1, int(bool(reverse1)),
                                              _ptr(X2), n2, _ptr(B), n_out, shift, s.real,
                                              s.imag)
        return self._check(st, "qtx_rgf_energy_convolution")

    def obc_lyapunov_fixed_point(self, b, batch, a, s_a, q, s_q, w, update, n_iter):
        """n_iter iterations of w <- q - a w a^dagger; see the C header."""
        st = lib().qtx_rgf_obc_lyapunov_fixed_point(self._h, b, batch, _ptr(a), s_a, _ptr(q),
                                                    s_q, _ptr(w), _ptr(update), n_iter)
        return self._check(st, "qtx_rgf_obc_lyapunov_fixed_point")

    def obc_lyapunov_doubling(self, b, batch, a, s_a, q, s_q, w, remaining, n_steps):
        """Doubling over the series of w = q - a w a^dagger; see the C header."""
        st = lib().qtx_rgf_obc_lyapunov_doubling(self._h, b, batch, _ptr(a), s_a, _ptr(q),
                                                 s_q, _ptr(w), _ptr(remaining), n_steps)
        return self._check(st, "qtx_rgf_obc_lyapunov_doubling")


def make_g_problem(energies_host, H, sigma_r, sigma_l, sigma_g, XR, XL=None,
                   XG=None, S=None, precision=QTX_FP64):
    """Problem structure for a G-type solve.

    energies_host: ctypes-compatible float64 numpy array (kept alive by the
    caller).  H, S: (diag, upper, lower) device tensors (upper/lower may be
    None).  sigma_*: (diag, upper, lower) per-energy device tensors.  XR, XL,
    XG: (diag, upper, lower) output tensors (XL/XG may be None).
    """
    n_e, n, b = sigma_r[0].shape[0], sigma_r[0].shape[1], sigma_r[0].shape[2]
    p = Problem()
    p.kind = QTX_KIND_G
    p.precision = precision
    p.n_blocks, p.block_size, p.n_energies = n, b, n_e
    p.energies = energies_host.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.H = _bt_in(*H)
    if S is not None:
        p.S = _bt_in(*S)
    p.sigma_r = _bt_in(*sigma_r)
    p.sigma_l = _bt_in(*(sigma_l or (None, None, None)))
    p.sigma_g = _bt_in(*(sigma_g or (None, None, None)))
    p.XR = _bt_out(*XR)
    p.XL = _bt_out(*(XL or (None, None, None)))
    p.XG = _bt_out(*(XG or (None, None, None)))
    p.status = -1
    return p


def make_w_problem(V, P_r, P_l, P_g, XR, XL=None, XG=None, WR_diag=None,
                   precision=QTX_FP64):
    n_e, n, b = P_r[0].shape[0], P_r[0].shape[1], P_r[0].shape[2]
    p = Problem()
    p.kind = QTX_KIND_W
    p.precision = precision
    p.n_blocks, p.block_size, p.n_energies = n, b, n_e
    p.V = _bt_in(*V)
    p.P_r = _bt_in(*P_r)
    p.P_l = _bt_in(*(P_l or (None, None, None)))
    p.P_g = _bt_in(*(P_g or (None, None, None)))
    p.XR = _bt_out(*XR)
    p.XL = _bt_out(*(XL or (None, None, None)))
    p.XG = _bt_out(*(XG or (None, None, None)))
    p.WR_diag = _ptr(WR_diag)
    p.status = -1
    return p
