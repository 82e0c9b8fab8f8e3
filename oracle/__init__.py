"""CPU oracle for the regularised KKT hot path (TEST INFRASTRUCTURE ONLY).

Plain FP64 reference of everything the GPU library computes: the KKT
assembly (``oracle.assemble``, numpy), and the symbolic analysis, the
pivot-free LDL^T and the solves (``ncl_oracle.c``, plain C).  Only the
tests, the smoke check and the benchmark's CPU-baseline leg use it; the
product path never imports, links or runs anything here.  It shares no
code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import assemble as _asm

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libncl_oracle.so")
# The same C built with fused multiply-add contraction (FMA is allowed on
# both sides of every comparison): the difference between the two builds'
# factors measures how much an entry depends on the rounding of its own
# recurrence, which a perturbation of K cannot show where large terms cancel
# exactly (the pivot of a complementarity row can be 1e-9 of the terms that
# form it).
_SO_FMA = os.path.join(_HERE, "libncl_oracle_fma.so")
_libs = {}

DEFAULT_RELAX = (16, 1, 4)      # maxw, znum, zden


def host_has_fma() -> bool:
    try:
        with open("/proc/cpuinfo") as f:
            return any(line.startswith("flags") and " fma " in line + " " for line in f)
    except OSError:
        return False


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, OpenMP), and its FMA build where the host
    has FMA."""
    src = os.path.join(_HERE, "ncl_oracle.c")
    base = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99"]
    if force or not os.path.exists(_SO):
        subprocess.check_call(base + ["-ffp-contract=off", "-o", _SO, src, "-lm"])
    if host_has_fma() and (force or not os.path.exists(_SO_FMA)):
        subprocess.check_call(base + ["-mfma", "-ffp-contract=fast", "-o", _SO_FMA, src, "-lm"])
    return _SO


def _load(fma=False):
    if fma not in _libs:
        so = _SO_FMA if fma else _SO
        if not os.path.exists(so):
            build(force=False)
        if not os.path.exists(so):
            raise RuntimeError("the FMA build of the oracle needs a host with FMA")
        L = ctypes.CDLL(so)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        L.oracle_symbolic.argtypes = [i64, P, P, i32, P, i32, i32, i32, P, ctypes.POINTER(P)]
        L.oracle_symbolic.restype = ctypes.c_int
        for f in ("oracle_N", "oracle_nnzl", "oracle_nsuper", "oracle_npanel"):
            getattr(L, f).argtypes = [P]
            getattr(L, f).restype = i64
        L.oracle_get_symbolic.argtypes = [P] * 9
        L.oracle_get_symbolic.restype = None
        L.oracle_factor.argtypes = [P, P, P, P, i32]
        L.oracle_factor.restype = ctypes.c_int
        L.oracle_get_numeric.argtypes = [P, P, P, P]
        L.oracle_get_numeric.restype = None
        L.oracle_solve.argtypes = [P, P, P, i32, i64]
        L.oracle_solve.restype = ctypes.c_int
        L.oracle_free.argtypes = [P]
        L.oracle_free.restype = None
        _libs[fma] = L
    return _libs[fma]


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def lower_csc(rows, cols, vals, N):
    """CSC of the lower triangle (rows sorted within each column)."""
    order = np.lexsort((rows, cols))
    r, c, v = rows[order], cols[order], vals[order]
    colptr = np.zeros(N + 1, np.int64)
    np.add.at(colptr, c + 1, 1)
    colptr = np.cumsum(colptr)
    return colptr, r.astype(np.int32), np.ascontiguousarray(v, np.float64)


class Factor:
    """Symbolic analysis plus (after ``factor``) the numeric LDL^T.

    ``perm``: a caller's elimination order (new -> layout index) in place of
    minimum degree; it must keep every block's columns inside the block and
    the border in layout order.  ``fma``: use the build with fused
    multiply-add contraction (same arithmetic, other rounding)."""

    def __init__(self, N, colptr, rowind, block_off, relax=DEFAULT_RELAX, perm=None, fma=False):
        self._fma = bool(fma)
        L = _load(self._fma)
        self.N = int(N)
        self.colptr = np.ascontiguousarray(colptr, np.int64)
        self.rowind = np.ascontiguousarray(rowind, np.int32)
        self.block_off = np.ascontiguousarray(block_off, np.int64)
        nblk = self.block_off.shape[0] - 1
        h = ctypes.c_void_p()
        up = None if perm is None else np.ascontiguousarray(perm, np.int32)
        rc = L.oracle_symbolic(self.N, _ptr(self.colptr), _ptr(self.rowind), nblk, _ptr(self.block_off),
                               int(relax[0]), int(relax[1]), int(relax[2]), _ptr(up), ctypes.byref(h))
        if rc != 0:
            raise RuntimeError(f"oracle_symbolic failed: {rc}")
        self._h = h
        self.nnzl = int(L.oracle_nnzl(h))
        self.nsuper = int(L.oracle_nsuper(h))
        npan = int(L.oracle_npanel(h))
        self.perm = np.empty(self.N, np.int32)
        self.parent = np.empty(self.N, np.int32)
        self.colcount = np.empty(self.N, np.int64)
        self.lp = np.empty(self.N + 1, np.int64)
        self.li = np.empty(max(self.nnzl, 1), np.int32)
        self.sup = np.empty(self.nsuper + 1, np.int64)
        self.srp = np.empty(self.nsuper + 1, np.int64)
        self.sri = np.empty(max(npan, 1), np.int32)
        L.oracle_get_symbolic(h, _ptr(self.perm), _ptr(self.parent), _ptr(self.colcount), _ptr(self.lp),
                              _ptr(self.li), _ptr(self.sup), _ptr(self.srp), _ptr(self.sri))
        self.li = self.li[:self.nnzl]
        self.sri = self.sri[:npan]
        self.factored = False

    @classmethod
    def from_network(cls, net, relax=DEFAULT_RELAX, perm=None):
        z = np.zeros(_asm.Positions(net).N)
        r, c, v, pos = _asm.assemble(net, z + 1.0, z + 1.0)
        colptr, rowind, _ = lower_csc(r, c, v, pos.N)
        f = cls(pos.N, colptr, rowind, np.array(pos.block_off, np.int64), relax, perm)
        f.pos = pos
        return f

    def factor(self, colptr, rowind, vals, nthreads=1):
        L = _load(self._fma)
        vals = np.ascontiguousarray(vals, np.float64)
        rc = L.oracle_factor(self._h, _ptr(np.ascontiguousarray(colptr, np.int64)),
                             _ptr(np.ascontiguousarray(rowind, np.int32)), _ptr(vals), int(nthreads))
        self.lx = np.empty(max(self.nnzl, 1), np.float64)
        self.d = np.empty(self.N, np.float64)
        inertia = np.empty(4, np.int64)
        L.oracle_get_numeric(self._h, _ptr(self.lx), _ptr(self.d), _ptr(inertia))
        self.lx = self.lx[:self.nnzl]
        self.inertia = tuple(int(x) for x in inertia[:3])
        self.first_bad = int(inertia[3])
        self.factored = True
        return rc

    def solve(self, b):
        """x = K^{-1} b; b is (N,) or (nrhs, N) in layout order."""
        L = _load(self._fma)
        b2 = np.ascontiguousarray(np.atleast_2d(b), np.float64)
        x = np.empty_like(b2)
        rc = L.oracle_solve(self._h, _ptr(b2), _ptr(x), b2.shape[0], self.N)
        if rc != 0:
            raise RuntimeError(f"oracle_solve failed: {rc}")
        return x.reshape(np.shape(b))

    def L_csc(self):
        """Unit-lower L (strict part) as scipy CSC in the permuted numbering."""
        import scipy.sparse as sp
        return sp.csc_matrix((self.lx, self.li, self.lp), shape=(self.N, self.N))

    def __del__(self):
        try:
            if self._h:
                _load(self._fma).oracle_free(self._h)
                self._h = None
        except Exception:
            pass


def kkt(net, z, sigma, diag_shift=True):
    """Assemble K for a state: returns (colptr, rowind, vals, pos) lower CSC in layout order."""
    r, c, v, pos = _asm.assemble(net, z, sigma, diag_shift=diag_shift)
    colptr, rowind, vals = lower_csc(r, c, v, pos.N)
    return colptr, rowind, vals, pos


def spmv(colptr, rowind, vals, x):
    """y = K x for the symmetric K given by its lower CSC (x: (N,) or (nrhs, N))."""
    import scipy.sparse as sp
    N = colptr.shape[0] - 1
    Lw = sp.csc_matrix((vals, rowind, colptr), shape=(N, N))
    full = Lw + Lw.T - sp.diags(Lw.diagonal())
    xt = np.atleast_2d(x)
    y = (full @ xt.T).T
    return y.reshape(np.shape(x))


def backward_error(colptr, rowind, vals, x, b):
    """Normwise backward error max over columns of
    ||b - Kx||_inf / (||K||_inf ||x||_inf + ||b||_inf)."""
    import scipy.sparse as sp
    N = colptr.shape[0] - 1
    Lw = sp.csc_matrix((vals, rowind, colptr), shape=(N, N))
    full = Lw + Lw.T - sp.diags(Lw.diagonal())
    knorm = abs(full).sum(axis=1).max()
    X = np.atleast_2d(x)
    B = np.atleast_2d(b)
    R = B - (full @ X.T).T
    eta = np.abs(R).max(axis=1) / (knorm * np.abs(X).max(axis=1) + np.abs(B).max(axis=1))
    return float(eta.max())


def componentwise_backward_error(colptr, rowind, vals, x, b):
    """Componentwise (Oettli-Prager) backward error, max over columns of
    max_i |b - Kx|_i / (|K| |x| + |b|)_i.  A row whose denominator is zero
    counts 0 when its residual is zero and +inf otherwise.  Unlike the
    normwise error it sees a wrong component in a row whose own scale is
    far below ||K|| ||x||."""
    import scipy.sparse as sp
    N = colptr.shape[0] - 1
    Lw = sp.csc_matrix((vals, rowind, colptr), shape=(N, N))
    full = Lw + Lw.T - sp.diags(Lw.diagonal())
    X = np.atleast_2d(x)
    B = np.atleast_2d(b)
    R = np.abs(B - (full @ X.T).T)
    den = (abs(full) @ np.abs(X).T).T + np.abs(B)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(den > 0, R / np.where(den > 0, den, 1.0), np.where(R > 0, np.inf, 0.0))
    return float(q.max())
