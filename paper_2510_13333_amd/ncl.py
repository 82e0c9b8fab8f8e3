"""ctypes binding of libnclkkt (include/ncl_kkt.h).

Argument marshalling only: every step of assembly, factorisation and solve
runs in the library's HIP kernels.  PyTorch provides device memory (the
workspace and the vectors) and the current stream.  The library must have
been built (``paper_2510_13333_amd._build.build()``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libnclkkt.so")
_lib = None

NCL_PVPQ = 1
NCL_SCREEN = 2
NCL_AGC = 4
NCL_TRACE_W = 9

# kernel kinds (NCL_K_* of ncl_kkt.h), in enum order
KERNELS = ["assemble", "values", "fac_gather", "fac_diag", "fac_rows", "border_schur", "border_sum",
           "border_factor", "status_init", "status", "sol_load", "sol_fwd_gather", "sol_fwd_diag", "sol_bpart",
           "sol_border", "sol_bwd_border", "sol_bwd", "sol_store", "residual", "max_step", "interleave",
           "berr_rows", "berr_border", "berr_final"]

STATUS = {0: "ok", -1: "invalid argument", -2: "host allocation failed", -3: "HIP runtime error",
          -4: "call out of order", -5: "zero pivot", -6: "pivot of the wrong sign (inertia)",
          -7: "non-finite pivot", -8: "Newton method did not converge"}


class NclError(RuntimeError):
    def __init__(self, where, code):
        super().__init__(f"{where}: {STATUS.get(code, code)} ({code})")
        self.code = code


class _Network(ctypes.Structure):
    _fields_ = [("nbus", ctypes.c_int32), ("nbranch", ctypes.c_int32), ("ngen", ctypes.c_int32),
                ("ncont", ctypes.c_int32), ("br_from", ctypes.c_void_p), ("br_to", ctypes.c_void_p),
                ("gen_bus", ctypes.c_void_p), ("outage", ctypes.c_void_p), ("br_r", ctypes.c_void_p),
                ("br_x", ctypes.c_void_p), ("gen_c2", ctypes.c_void_p), ("flags", ctypes.c_uint32),
                ("gen_alpha", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("relax_maxw", ctypes.c_int32), ("relax_znum", ctypes.c_int32), ("relax_zden", ctypes.c_int32),
                ("ordering", ctypes.c_int32), ("user_perm", ctypes.c_void_p)]


NCL_ORDER_MD, NCL_ORDER_USER = 0, 1


NCL_NO_SHIFT = 1


class _Point(ctypes.Structure):
    _fields_ = [("z", ctypes.c_void_p), ("sigma", ctypes.c_void_p), ("rho", ctypes.c_double),
                ("flags", ctypes.c_uint32)]


class _Nlp(ctypes.Structure):
    _fields_ = [("pd", ctypes.c_void_p), ("qd_ratio", ctypes.c_double), ("mu", ctypes.c_double),
                ("rho", ctypes.c_double), ("vmin", ctypes.c_double), ("vmax", ctypes.c_double),
                ("qmax", ctypes.c_double), ("pmax", ctypes.c_double), ("smax2", ctypes.c_double),
                ("eps", ctypes.c_double)]


class NewtonOpts(ctypes.Structure):
    _fields_ = [("step_tol", ctypes.c_double), ("floor_tol", ctypes.c_double), ("maxit", ctypes.c_int32),
                ("from_default", ctypes.c_int32), ("iterations", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("dw_last", ctypes.c_double)]


class _IpmProblem(ctypes.Structure):
    _fields_ = [("pd", ctypes.c_void_p), ("lo", ctypes.c_void_p), ("hi", ctypes.c_void_p), ("y_n", ctypes.c_void_p),
                ("qd_ratio", ctypes.c_double), ("qmax", ctypes.c_double), ("pmax", ctypes.c_double),
                ("smax2", ctypes.c_double), ("eps", ctypes.c_double), ("mu", ctypes.c_double), ("rho", ctypes.c_double),
                ("pg0", ctypes.c_void_p), ("vm0", ctypes.c_void_p)]


class _IpmState(ctypes.Structure):
    _fields_ = [("z", ctypes.c_void_p), ("rt", ctypes.c_void_p), ("s", ctypes.c_void_p), ("zl", ctypes.c_void_p),
                ("zu", ctypes.c_void_p)]


class _IpmDirection(ctypes.Structure):
    _fields_ = [("dz", ctypes.c_void_p), ("drt", ctypes.c_void_p), ("ds", ctypes.c_void_p),
                ("dzl", ctypes.c_void_p), ("dzu", ctypes.c_void_p)]


class InertiaOpts(ctypes.Structure):
    _fields_ = [("dw_last", ctypes.c_double), ("nfactor", ctypes.c_int32), ("pad", ctypes.c_int32)]


class SolveOpts(ctypes.Structure):
    """Options of the NCL solve (ncl_solve_opts); the defaults below."""
    _fields_ = [("tol", ctypes.c_double), ("mu_min", ctypes.c_double), ("mu0", ctypes.c_double),
                ("mu_warm", ctypes.c_double), ("kappa_eps", ctypes.c_double), ("kappa_mu", ctypes.c_double),
                ("theta_mu", ctypes.c_double), ("tau_min", ctypes.c_double), ("eta0", ctypes.c_double),
                ("eta_shrink", ctypes.c_double), ("rho_grow", ctypes.c_double), ("rho_max", ctypes.c_double),
                ("max_inner", ctypes.c_int32), ("max_outer", ctypes.c_int32), ("trace", ctypes.c_void_p),
                ("trace_len", ctypes.c_int32), ("pad", ctypes.c_int32)]

    def __init__(self, trace=None, **kw):
        """trace: an optional float64 numpy array (n, NCL_TRACE_W) that the
        solve fills with its iteration log (kept alive by this object)."""
        d = dict(tol=1e-6, mu_min=1e-7, mu0=0.1, mu_warm=1e-5, kappa_eps=10.0, kappa_mu=0.2, theta_mu=1.5,
                 tau_min=0.99, eta0=1e-2, eta_shrink=10.0, rho_grow=10.0, rho_max=1e12, max_inner=300, max_outer=30)
        d.update(kw)
        super().__init__(**d)
        self._trace = trace
        if trace is not None:
            if trace.dtype != np.float64 or trace.ndim != 2 or trace.shape[1] != NCL_TRACE_W or \
                    not trace.flags["C_CONTIGUOUS"]:
                raise ValueError("trace must be a contiguous float64 array of shape (n, NCL_TRACE_W)")
            self.trace = trace.ctypes.data_as(ctypes.c_void_p)
            self.trace_len = trace.shape[0]


class _SolveReport(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer", ctypes.c_int32), ("inner", ctypes.c_int32),
                ("factorizations", ctypes.c_int32), ("rho", ctypes.c_double), ("mu", ctypes.c_double),
                ("r_inf", ctypes.c_double), ("kkt_err", ctypes.c_double)]


class _SolveState(ctypes.Structure):
    _fields_ = [("z", ctypes.c_void_p), ("rt", ctypes.c_void_p), ("s", ctypes.c_void_p), ("zl", ctypes.c_void_p),
                ("zu", ctypes.c_void_p), ("y_n", ctypes.c_void_p)]


class Report(ctypes.Structure):
    _fields_ = [("npos", ctypes.c_int64), ("nneg", ctypes.c_int64), ("nzero", ctypes.c_int64),
                ("first_bad", ctypes.c_int64), ("min_absd", ctypes.c_double), ("max_absd", ctypes.c_double),
                ("status", ctypes.c_int32), ("solvable", ctypes.c_int32), ("nnonfinite", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def library_path() -> str:
    return _SO


def load():
    """Load libnclkkt.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        raise RuntimeError(f"{_SO} is missing: build it with paper_2510_13333_amd._build.build()")
    L = ctypes.CDLL(_SO)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "ncl_kkt_analyze": ([P, P, pp], ctypes.c_int),
        "ncl_kkt_analyze_pattern": ([i64, i32, P, P, P, P, P, pp], ctypes.c_int),
        "ncl_kkt_analyze_batch": ([P, i32, P, i32, pp], ctypes.c_int),
        "ncl_kkt_instances": ([P, P], ctypes.c_int),
        "ncl_kkt_instance": ([P, i32, P, P, P, P, P], ctypes.c_int),
        "ncl_kkt_dims": ([P, P, P, P, P, P, P], ctypes.c_int),
        "ncl_kkt_symbolic": ([P, P, P, P, P, P, P, P, P], ctypes.c_int),
        "ncl_kkt_pattern": ([P, P, P], ctypes.c_int),
        "ncl_kkt_workspace_bytes": ([P, i32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ncl_kkt_bind_workspace": ([P, P, ctypes.c_size_t, i32, P], ctypes.c_int),
        "ncl_kkt_assemble": ([P, P, P], ctypes.c_int),
        "ncl_kkt_set_values": ([P, P, P], ctypes.c_int),
        "ncl_kkt_get_values": ([P, P, P], ctypes.c_int),
        "ncl_kkt_factor": ([P, P], ctypes.c_int),
        "ncl_kkt_factor_blocks": ([P, P], ctypes.c_int),
        "ncl_kkt_factor_border": ([P, P], ctypes.c_int),
        "ncl_kkt_info": ([P, P, P], ctypes.c_int),
        "ncl_kkt_get_factors": ([P, P, P, P], ctypes.c_int),
        "ncl_kkt_solve": ([P, P, P, i32, i64, P], ctypes.c_int),
        "ncl_kkt_factor_solve": ([P, P, P, i32, i64, P], ctypes.c_int),
        "ncl_kkt_solve_adjoint": ([P, P, P, i32, i64, P], ctypes.c_int),
        "ncl_kkt_backward_error": ([P, P, P, i32, i64, P, P], ctypes.c_int),
        "ncl_kkt_refine": ([P, P, P, i32, i64, P], ctypes.c_int),
        "ncl_kkt_backward_error_noalloc": ([P, P, P, i32, i64, P, P], ctypes.c_int),
        "ncl_kkt_destroy": ([P], None),
        "ncl_kernel_name": ([ctypes.c_int], ctypes.c_char_p),
        "ncl_kkt_kernel_model": ([P, i32, P, P], ctypes.c_int),
        "ncl_kkt_profile": ([P, i32], ctypes.c_int),
        "ncl_kkt_profile_stride": ([P, i32], ctypes.c_int),
        "ncl_kkt_profile_read": ([P, P, P], ctypes.c_int),
        "ncl_kkt_residual": ([P, P, P, P, P, P], ctypes.c_int),
        "ncl_kkt_layout_kinds": ([P, P], ctypes.c_int),
        "ncl_kkt_max_step": ([P, P, P, P, ctypes.c_double, P, P], ctypes.c_int),
        "ncl_kkt_dispatch_newton": ([P, P, P, P, P, P], ctypes.c_int),
        "ncl_kkt_dispatch_outputs": ([P, P, P, P, P], ctypes.c_int),
        "ncl_kkt_dispatch_vjp": ([P, P, P, P, P, P, P, P], ctypes.c_int),
        "ncl_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "ncl_stream_copy": ([P, P, i64, P], ctypes.c_int),
        "ncl_kkt_ipm_sigma": ([P, P, P, P, P], ctypes.c_int),
        "ncl_kkt_ipm_rhs": ([P, P, P, P, P, P], ctypes.c_int),
        "ncl_kkt_ipm_recover": ([P, P, P, P, P, P], ctypes.c_int),
        "ncl_kkt_factor_inertia": ([P, P, P, ctypes.c_double, P, P, P], ctypes.c_int),
        "ncl_kkt_ipm_step": ([P, P, P, P, P, P, P], ctypes.c_int),
        "ncl_kkt_ncl_solve": ([P, P, P, P, P, P, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def stream_copy(src, dst):
    """dst[:] = src by the library's streaming copy kernel (device float64
    tensors of one even length)."""
    if src.numel() != dst.numel():
        raise ValueError("src and dst differ in length")
    _check("ncl_stream_copy", load().ncl_stream_copy(KKT._dev(src), KKT._dev(dst), int(src.numel()), _stream_ptr()))


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(where, rc):
    if rc != 0:
        raise NclError(where, rc)


def _stream_ptr():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _network_struct(net, keep):
    arrs = dict(br_from=np.ascontiguousarray(net.br_from, np.int32),
                br_to=np.ascontiguousarray(net.br_to, np.int32),
                gen_bus=np.ascontiguousarray(net.gen_bus, np.int32),
                outage=np.ascontiguousarray(net.outage, np.int32),
                br_r=np.ascontiguousarray(net.br_r, np.float64),
                br_x=np.ascontiguousarray(net.br_x, np.float64),
                gen_c2=np.ascontiguousarray(net.gen_c2, np.float64))
    agc = bool(getattr(net, "agc", False))
    if agc:
        arrs["gen_alpha"] = np.ascontiguousarray(net.gen_alpha, np.float64)
    keep.append(arrs)
    flags = ((NCL_PVPQ if getattr(net, "pvpq", False) else 0) | (NCL_SCREEN if getattr(net, "screen", False) else 0) |
             (NCL_AGC if agc else 0))
    return _Network(int(net.nb), int(net.nl), int(net.ng), int(arrs["outage"].shape[0]),
                    *[_np_ptr(arrs[k]) for k in ("br_from", "br_to", "gen_bus", "outage", "br_r", "br_x", "gen_c2")],
                    flags, _np_ptr(arrs["gen_alpha"]) if agc else None)


class KKT:
    """One analysed KKT pattern (ncl_kkt handle) and, once bound, its workspace.

    ``KKT(net)`` analyses one network; ``KKT(nets=[...])`` analyses a batch
    of independent networks in one handle (every launch then covers all of
    them; vectors are the instances' layout-order vectors concatenated).
    ``relax`` is one (maxw, znum, zden) triple, or with a batch optionally a
    list with one triple per instance.  ``perm`` (single network or
    pattern): a caller-given elimination order, new -> layout index
    (NCL_ORDER_USER); None takes minimum degree."""

    def __init__(self, net=None, *, relax=None, pattern=None, nets=None, perm=None):
        L = load()
        self._h = ctypes.c_void_p()
        self._keep = []
        opts = None
        if relax is not None and not (nets is not None and isinstance(relax, (list, tuple))
                                      and len(relax) and isinstance(relax[0], (list, tuple))):
            opts = _Opts(int(relax[0]), int(relax[1]), int(relax[2]), NCL_ORDER_MD, None)
        if perm is not None:
            if nets is not None:
                raise ValueError("perm is for a single network or pattern")
            pa = np.ascontiguousarray(perm, np.int32)
            self._keep.append(pa)
            if opts is None:
                opts = _Opts(0, 0, 0, NCL_ORDER_USER, None)
            opts.ordering = NCL_ORDER_USER
            opts.user_perm = _np_ptr(pa).value
        if nets is not None:
            nets = list(nets)
            arr = (_Network * len(nets))(*[_network_struct(n, self._keep) for n in nets])
            nopts = 0
            optp = None
            if opts is not None:
                optp, nopts = ctypes.byref(opts), 1
            elif relax is not None:
                oarr = (_Opts * len(nets))(*[_Opts(int(r[0]), int(r[1]), int(r[2]), NCL_ORDER_MD, None)
                                             for r in relax])
                self._keep.append(oarr)
                optp, nopts = oarr, len(nets)
            rc = L.ncl_kkt_analyze_batch(arr, len(nets), optp, nopts, ctypes.byref(self._h))
            _check("ncl_kkt_analyze_batch", rc)
        elif net is not None:
            s = _network_struct(net, self._keep)
            rc = L.ncl_kkt_analyze(ctypes.byref(s), ctypes.byref(opts) if opts else None, ctypes.byref(self._h))
            _check("ncl_kkt_analyze", rc)
        elif pattern is not None:
            N, block_off, colptr, rowind, is_primal = pattern
            block_off = np.ascontiguousarray(block_off, np.int64)
            colptr = np.ascontiguousarray(colptr, np.int64)
            rowind = np.ascontiguousarray(rowind, np.int32)
            is_primal = np.ascontiguousarray(is_primal, np.uint8)
            rc = L.ncl_kkt_analyze_pattern(int(N), int(block_off.shape[0] - 1), _np_ptr(block_off), _np_ptr(colptr),
                                           _np_ptr(rowind), _np_ptr(is_primal),
                                           ctypes.byref(opts) if opts else None, ctypes.byref(self._h))
            _check("ncl_kkt_analyze_pattern", rc)
        else:
            raise ValueError("need a network or a pattern")
        d = [ctypes.c_int64() for _ in range(6)]
        _check("ncl_kkt_dims", L.ncl_kkt_dims(self._h, *[ctypes.byref(x) for x in d]))
        self.N, self.nprimal, self.nnzK, self.nnzL, self.nsuper, self.npanel = (int(x.value) for x in d)
        self.ws = None
        self.nrhs_max = 0
        cnt = ctypes.c_int32()
        _check("ncl_kkt_instances", L.ncl_kkt_instances(self._h, ctypes.byref(cnt)))
        self.instances = []
        for i in range(cnt.value):
            c0, n, npr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
            nbk, nbd = ctypes.c_int32(), ctypes.c_int32()
            _check("ncl_kkt_instance", L.ncl_kkt_instance(self._h, i, ctypes.byref(c0), ctypes.byref(n),
                                                          ctypes.byref(npr), ctypes.byref(nbk), ctypes.byref(nbd)))
            self.instances.append(dict(col0=c0.value, N=n.value, nprimal=npr.value, nblk=nbk.value,
                                       nbd=nbd.value))

    # ------------------------------------------------------------ symbolic (host)
    def symbolic(self):
        L = load()
        out = dict(perm=np.empty(self.N, np.int32), etree=np.empty(self.N, np.int32),
                   colcount=np.empty(self.N, np.int64), super_ptr=np.empty(self.nsuper + 1, np.int64),
                   lcolptr=np.empty(self.N + 1, np.int64), lrowind=np.empty(max(self.nnzL, 1), np.int32),
                   srowptr=np.empty(self.nsuper + 1, np.int64), srowind=np.empty(max(self.npanel, 1), np.int32))
        _check("ncl_kkt_symbolic", L.ncl_kkt_symbolic(self._h, *[_np_ptr(out[k]) for k in (
            "perm", "etree", "colcount", "super_ptr", "lcolptr", "lrowind", "srowptr", "srowind")]))
        out["lrowind"] = out["lrowind"][:self.nnzL]
        out["srowind"] = out["srowind"][:self.npanel]
        return out

    def pattern(self):
        L = load()
        cp = np.empty(self.N + 1, np.int64)
        ri = np.empty(max(self.nnzK, 1), np.int32)
        _check("ncl_kkt_pattern", L.ncl_kkt_pattern(self._h, _np_ptr(cp), _np_ptr(ri)))
        return cp, ri[:self.nnzK]

    def workspace_bytes(self, nrhs_max=1):
        n = ctypes.c_size_t()
        _check("ncl_kkt_workspace_bytes", load().ncl_kkt_workspace_bytes(self._h, int(nrhs_max), ctypes.byref(n)))
        return int(n.value)

    # ------------------------------------------------------------ device
    def bind(self, nrhs_max=1, device="cuda"):
        import torch
        nbytes = self.workspace_bytes(nrhs_max)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = ws.data_ptr()
        off = (-base) % 256
        self.ws = ws
        _check("ncl_kkt_bind_workspace", load().ncl_kkt_bind_workspace(
            self._h, ctypes.c_void_p(base + off), ctypes.c_size_t(nbytes), int(nrhs_max), _stream_ptr()))
        self.nrhs_max = int(nrhs_max)
        return self

    @staticmethod
    def _dev(t, n=None):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise TypeError("expected a contiguous float64 CUDA tensor")
        if n is not None and t.numel() < n:
            raise ValueError("tensor too short")
        return ctypes.c_void_p(t.data_ptr())

    def assemble(self, z, sigma, rho, shift=True):
        """K at state (z, sigma); shift=False assembles without the diagonal-dominance shift."""
        pt = _Point(self._dev(z, self.N), self._dev(sigma, self.N), float(rho), 0 if shift else NCL_NO_SHIFT)
        self._pt = (z, sigma)
        _check("ncl_kkt_assemble", load().ncl_kkt_assemble(self._h, ctypes.byref(pt), _stream_ptr()))

    def set_values(self, vals):
        _check("ncl_kkt_set_values", load().ncl_kkt_set_values(self._h, self._dev(vals, self.nnzK), _stream_ptr()))

    def get_values(self):
        import torch
        out = torch.empty(self.nnzK, dtype=torch.float64, device=self.ws.device)
        _check("ncl_kkt_get_values", load().ncl_kkt_get_values(self._h, self._dev(out), _stream_ptr()))
        return out

    def factor(self):
        _check("ncl_kkt_factor", load().ncl_kkt_factor(self._h, _stream_ptr()))

    def factor_blocks(self):
        _check("ncl_kkt_factor_blocks", load().ncl_kkt_factor_blocks(self._h, _stream_ptr()))

    def factor_border(self):
        _check("ncl_kkt_factor_border", load().ncl_kkt_factor_border(self._h, _stream_ptr()))

    def info(self):
        rep = Report()
        _check("ncl_kkt_info", load().ncl_kkt_info(self._h, ctypes.byref(rep), _stream_ptr()))
        return rep.as_dict()

    def get_factors(self):
        lx = np.empty(max(self.nnzL, 1), np.float64)
        d = np.empty(self.N, np.float64)
        _check("ncl_kkt_get_factors", load().ncl_kkt_get_factors(self._h, _np_ptr(lx), _np_ptr(d), _stream_ptr()))
        return lx[:self.nnzL], d

    def _solve(self, fn, b, out=None):
        import torch
        b2 = b if b.dim() == 2 else b.reshape(1, -1)
        nrhs, ld = b2.shape
        if out is None:
            out = torch.empty_like(b2)
        _check(fn, getattr(load(), fn)(self._h, self._dev(b2), self._dev(out), int(nrhs), int(ld), _stream_ptr()))
        return out if b.dim() == 2 else out.reshape(-1)

    def _solve_ld(self, b, out, ld):
        """Solve nrhs columns stored ld apart (b, out: device tensors whose
        data start at column 0 of the first right-hand side)."""
        import torch  # noqa: F401
        nrhs = b.shape[0]
        _check("ncl_kkt_solve", load().ncl_kkt_solve(self._h, ctypes.c_void_p(b.data_ptr()),
                                                     ctypes.c_void_p(out.data_ptr()), int(nrhs), int(ld),
                                                     _stream_ptr()))
        return out

    def solve(self, b, out=None):
        """x = K^{-1} b; b is (N,) or (nrhs, N) float64 on the device, layout order."""
        return self._solve("ncl_kkt_solve", b, out)

    def factor_solve(self, b, out=None):
        """Factor the current values and solve, the border's factorisation
        overlapped with the blocks' forward substitution on a second stream."""
        return self._solve("ncl_kkt_factor_solve", b, out)

    def solve_adjoint(self, b, out=None):
        return self._solve("ncl_kkt_solve_adjoint", b, out)

    def backward_error(self, b, x, out=None, noalloc=False):
        """(eta, omega) per column, on the device (no synchronisation): a
        (nrhs, 2) float64 tensor, or written into ``out``.  noalloc: the
        library-held staging (ncl_kkt_backward_error_noalloc)."""
        import torch
        b2 = b if b.dim() == 2 else b.reshape(1, -1)
        x2 = x if x.dim() == 2 else x.reshape(1, -1)
        if b2.shape != x2.shape:
            raise ValueError("b and x differ in shape")
        if out is None:
            out = torch.empty((b2.shape[0], 2), dtype=torch.float64, device=b.device)
        fn = "ncl_kkt_backward_error_noalloc" if noalloc else "ncl_kkt_backward_error"
        _check(fn, getattr(load(), fn)(
            self._h, self._dev(b2), self._dev(x2), int(b2.shape[0]), int(b2.shape[1]), self._dev(out, 2 * b2.shape[0]),
            _stream_ptr()))
        return out

    def refine(self, b, x):
        """One step of iterative refinement of x (in place) on the stored factors."""
        b2 = b if b.dim() == 2 else b.reshape(1, -1)
        x2 = x if x.dim() == 2 else x.reshape(1, -1)
        if b2.shape != x2.shape:
            raise ValueError("b and x differ in shape")
        _check("ncl_kkt_refine", load().ncl_kkt_refine(self._h, self._dev(b2), self._dev(x2), int(b2.shape[0]),
                                                      int(b2.shape[1]), _stream_ptr()))
        return x

    # ------------------------------------------------------------ dispatch map
    def layout_kinds(self):
        """Kind code (NCL_L_*) of every global column, host uint8 array."""
        out = np.empty(self.N, np.uint8)
        _check("ncl_kkt_layout_kinds", load().ncl_kkt_layout_kinds(self._h, _np_ptr(out)))
        return out

    @staticmethod
    def _nlp(pd, p):
        return _Nlp(ctypes.c_void_p(pd.data_ptr()), float(p["qd_ratio"]), float(p["mu"]), float(p["rho"]),
                    float(p["vmin"]), float(p["vmax"]), float(p["qmax"]), float(p["pmax"]), float(p["smax2"]),
                    float(p["eps"]))

    def residual(self, z, pd, p, F=None, sigma=None):
        """F(z; pd) and sigma of the dispatch map (device tensors); p: dict of ncl_nlp fields."""
        import torch
        F = torch.empty_like(z) if F is None else F
        sigma = torch.empty_like(z) if sigma is None else sigma
        self._dev(pd)
        q = self._nlp(pd, p)
        _check("ncl_kkt_residual", load().ncl_kkt_residual(self._h, ctypes.byref(q), self._dev(z, self.N),
                                                           self._dev(F, self.N), self._dev(sigma, self.N),
                                                           _stream_ptr()))
        return F, sigma

    def max_step(self, z, dz, pd, p, tau, out):
        """Writes the fraction-to-boundary step length into the 1-element device tensor out."""
        self._dev(pd)
        q = self._nlp(pd, p)
        _check("ncl_kkt_max_step", load().ncl_kkt_max_step(self._h, ctypes.byref(q), self._dev(z, self.N),
                                                           self._dev(dz, self.N), float(tau), self._dev(out),
                                                           _stream_ptr()))
        return out

    def dispatch_newton(self, pd, p, z, work, opts):
        """Newton solve of the dispatch map in the library (z in/out, work:
        7 N + 8 doubles on the device, opts: NewtonOpts, updated)."""
        self._dev(pd)
        q = self._nlp(pd, p)
        _check("ncl_kkt_dispatch_newton", load().ncl_kkt_dispatch_newton(
            self._h, ctypes.byref(q), self._dev(z, self.N), self._dev(work, 7 * self.N + 8), ctypes.byref(opts),
            _stream_ptr()))
        return z

    def dispatch_outputs(self, z, phi, pg=None):
        _check("ncl_kkt_dispatch_outputs", load().ncl_kkt_dispatch_outputs(
            self._h, self._dev(z, self.N), self._dev(phi), None if pg is None else self._dev(pg), _stream_ptr()))
        return phi, pg

    def dispatch_vjp(self, pd, p, z, gphi, gpg, gpd, work):
        """gpd = the load cotangent of (gphi, gpg) at the solution z (one
        adjoint solve on the stored factors; work: 2 N doubles)."""
        self._dev(pd)
        q = self._nlp(pd, p)
        _check("ncl_kkt_dispatch_vjp", load().ncl_kkt_dispatch_vjp(
            self._h, ctypes.byref(q), self._dev(z, self.N), self._dev(gphi), None if gpg is None else self._dev(gpg),
            self._dev(gpd), self._dev(work, 2 * self.N), _stream_ptr()))
        return gpd

    # ------------------------------------------------------------ IPM step
    def _ipm(self, prob, state):
        """Marshal the IPM problem (dict: pd, lo, hi, y_n device tensors and
        the scalars qd_ratio, qmax, pmax (default 8), smax2, eps, mu, rho, and
        for screening networks pg0, vm0 device tensors) and state (dict: z,
        rt, s, zl, zu device tensors)."""
        p = _IpmProblem(self._dev(prob["pd"]), self._dev(prob["lo"], self.N), self._dev(prob["hi"], self.N),
                        self._dev(prob["y_n"], self.N), float(prob["qd_ratio"]), float(prob["qmax"]),
                        float(prob.get("pmax", 8.0)), float(prob["smax2"]), float(prob["eps"]), float(prob["mu"]),
                        float(prob["rho"]), None if prob.get("pg0") is None else self._dev(prob["pg0"]),
                        None if prob.get("vm0") is None else self._dev(prob["vm0"]))
        st = _IpmState(*[self._dev(state[k], self.N) for k in ("z", "rt", "s", "zl", "zu")])
        return p, st

    def _ipm_dir(self, d):
        return _IpmDirection(*[self._dev(d[k], self.N) for k in ("dz", "drt", "ds", "dzl", "dzu")])

    def ipm_sigma(self, prob, state, out):
        p, st = self._ipm(prob, state)
        _check("ncl_kkt_ipm_sigma", load().ncl_kkt_ipm_sigma(self._h, ctypes.byref(p), ctypes.byref(st),
                                                             self._dev(out, self.N), _stream_ptr()))
        return out

    def ipm_rhs(self, prob, state, out, work):
        """The reduced right-hand side; J'y from the K values held (assembled at state z); work: 2 N doubles."""
        p, st = self._ipm(prob, state)
        _check("ncl_kkt_ipm_rhs", load().ncl_kkt_ipm_rhs(self._h, ctypes.byref(p), ctypes.byref(st),
                                                         self._dev(out, self.N), self._dev(work, 2 * self.N),
                                                         _stream_ptr()))
        return out

    def ipm_recover(self, prob, state, dz, d):
        """Writes d["drt"], d["ds"], d["dzl"], d["dzu"] from dz = (dw, dy)."""
        p, st = self._ipm(prob, state)
        dd = _IpmDirection(None, *[self._dev(d[k], self.N) for k in ("drt", "ds", "dzl", "dzu")])
        _check("ncl_kkt_ipm_recover", load().ncl_kkt_ipm_recover(self._h, ctypes.byref(p), ctypes.byref(st),
                                                                 self._dev(dz, self.N), ctypes.byref(dd),
                                                                 _stream_ptr()))
        return d

    def factor_inertia(self, z, sigma, rho, opts, work):
        """Inertia-corrected factorisation at (z, sigma); opts: InertiaOpts (updated); work: N doubles."""
        _check("ncl_kkt_factor_inertia", load().ncl_kkt_factor_inertia(
            self._h, self._dev(z, self.N), self._dev(sigma, self.N), float(rho), ctypes.byref(opts),
            self._dev(work, self.N), _stream_ptr()))
        return opts

    def ipm_step(self, prob, state, d, opts, work):
        """One IPM direction into d (dict of device tensors dz, drt, ds, dzl,
        dzu); opts: InertiaOpts (updated); work: 3 N doubles."""
        p, st = self._ipm(prob, state)
        dd = self._ipm_dir(d)
        _check("ncl_kkt_ipm_step", load().ncl_kkt_ipm_step(self._h, ctypes.byref(p), ctypes.byref(st),
                                                           ctypes.byref(dd), ctypes.byref(opts),
                                                           self._dev(work, 3 * self.N), _stream_ptr()))
        return d

    def ncl_solve(self, prob, state, opts=None, work=None):
        """The NCL method end to end (ncl_kkt_ncl_solve).  prob: as for the
        IPM step (its y_n and mu are not read; rho is the first penalty);
        state: dict of device tensors z, rt, s, zl, zu, y_n, updated in place
        to the last iterate; work: 17 N + 64 doubles (allocated if None).
        Returns the report as a dict."""
        import torch
        if work is None:
            work = torch.empty(17 * self.N + 64, dtype=torch.float64, device=state["z"].device)
        prob = dict(prob)
        prob.setdefault("y_n", state["y_n"])
        prob.setdefault("mu", 0.1)
        p, _ = self._ipm(prob, state)
        s = _SolveState(*[self._dev(state[k], self.N) for k in ("z", "rt", "s", "zl", "zu", "y_n")])
        o = opts if opts is not None else SolveOpts()
        r = _SolveReport()
        _check("ncl_kkt_ncl_solve", load().ncl_kkt_ncl_solve(self._h, ctypes.byref(p), ctypes.byref(s),
                                                             ctypes.byref(o), ctypes.byref(r),
                                                             self._dev(work, 17 * self.N + 64), _stream_ptr()))
        return {f: getattr(r, f) for f, _ in r._fields_}

    # ------------------------------------------------------------ measurement
    @staticmethod
    def kernel_name(kind):
        n = load().ncl_kernel_name(int(kind))
        return n.decode() if n else None

    def kernel_model(self, kind):
        """(launches, algorithmic bytes) of one kernel kind per step."""
        la, by = ctypes.c_int64(), ctypes.c_int64()
        _check("ncl_kkt_kernel_model", load().ncl_kkt_kernel_model(self._h, int(kind), ctypes.byref(la),
                                                                   ctypes.byref(by)))
        return la.value, by.value

    def profile(self, kind):
        """Bracket later launches of one kernel kind with HIP events (-1 stops)."""
        _check("ncl_kkt_profile", load().ncl_kkt_profile(self._h, int(kind)))

    def profile_stride(self, stride):
        """Bracket only every stride-th launch of the profiled kind."""
        _check("ncl_kkt_profile_stride", load().ncl_kkt_profile_stride(self._h, int(stride)))

    def profile_read(self):
        """(bracketed launches, their summed event time in ms)."""
        n, ms = ctypes.c_int64(), ctypes.c_double()
        _check("ncl_kkt_profile_read", load().ncl_kkt_profile_read(self._h, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def __del__(self):
        try:
            if self._h:
                load().ncl_kkt_destroy(self._h)
                self._h = ctypes.c_void_p()
        except Exception:
            pass
