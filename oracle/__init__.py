"""FPE oracle — test infrastructure only.

A plain CPU reference (``fpe_oracle.c``) for the evaluation phase of the Fast
Polynomial Evaluator (arXiv 2211.06320, Algorithm A_p), plus the compensated
Horner evaluation of the full polynomial.  Only ``tests/``, the smoke check and
the CPU-baseline leg of ``bench.py`` may import this package; the product
library (``paper_2211_06320_amd``) never does, and the two share no code.

``build()`` compiles the C source with gcc; ``lib()`` loads the result (and
builds it if it is missing).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fpe_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_LIB = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build() -> str:
    """Compile the oracle (contraction off: the error-free transforms need it)."""
    tmp = _SO + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-pthread", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build()
    L = ctypes.CDLL(_SO)
    L.ora_scale1.restype = ctypes.c_int64
    L.ora_scale1.argtypes = [ctypes.c_double, ctypes.c_double]
    L.ora_scale.argtypes = [_f64p, ctypes.c_int64, _i64p]
    L.ora_precondition.restype = ctypes.c_void_p
    L.ora_precondition.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int32]
    L.ora_precondition_offset.restype = ctypes.c_void_p
    L.ora_precondition_offset.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int64]
    L.ora_plan_free.argtypes = [ctypes.c_void_p]
    L.ora_plan_info.argtypes = [ctypes.c_void_p, _i64p]
    L.ora_plan_hull.argtypes = [ctypes.c_void_p, _i64p, _i64p]
    L.ora_plan_good.argtypes = [ctypes.c_void_p, _u8p]
    L.ora_plan_scales.argtypes = [ctypes.c_void_p, _i64p]
    L.ora_eval.argtypes = [ctypes.c_void_p, _f64p, ctypes.c_int64, _f64p, _i64p, _i64p, _i64p,
                           _i64p, _f64p, _i64p, _f64p, _f64p, ctypes.c_int]
    L.ora_eval_deriv.argtypes = [ctypes.c_void_p, _f64p, ctypes.c_int64, _f64p, _i64p, _f64p, _i64p,
                                 _f64p, _i64p, _f64p, _i64p, ctypes.c_int]
    L.ora_horner.argtypes = [_f64p, ctypes.c_int64, _f64p, ctypes.c_int64, _f64p, _i64p, ctypes.c_int]
    L.ora_adjoint_coef.argtypes = [ctypes.c_void_p, _f64p, _f64p, ctypes.c_int64, ctypes.c_int64,
                                   _f64p, _i64p, _f64p, _i64p]
    L.ora_absum.argtypes = [_f64p, ctypes.c_int64, _f64p, ctypes.c_int64, _f64p, _i64p, ctypes.c_int]
    L.ora_eval_fp64.argtypes = [ctypes.c_void_p, _f64p, ctypes.c_int64, _f64p, _i64p, ctypes.c_int]
    L.ora_level_sets.argtypes = [ctypes.c_void_p, _f64p, _f64p, ctypes.c_int64, _f64p, _f64p, _f64p]
    L.ora_cancel_bound.argtypes = [ctypes.c_void_p, _f64p, _f64p, _f64p, _i64p, ctypes.c_int64,
                                   ctypes.POINTER(ctypes.c_int32)]
    _LIB = L
    return L


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _as_ri(c: np.ndarray) -> np.ndarray:
    """complex128 array -> contiguous float64 view (re, im interleaved)."""
    c = np.ascontiguousarray(np.asarray(c, dtype=np.complex128))
    return c.view(np.float64)


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


def scale(c) -> np.ndarray:
    """s(a) = 1 + floor(log2|a|) exactly; INT64_MIN for a == 0 (Section 2.3)."""
    ri = _as_ri(np.atleast_1d(c))
    out = np.empty(ri.shape[0] // 2, np.int64)
    lib().ora_scale(_ptr(ri, _f64p), out.shape[0], _ptr(out, _i64p))
    return out


NEG_INF = np.iinfo(np.int64).min


@dataclass
class PlanInfo:
    d: int
    v: int        # first nonzero index (-1 when P == 0)
    dt: int       # last nonzero index
    n_hull: int
    n_good: int
    T: int        # p + s(d_eff) + 3
    p: int


class OraclePlan:
    """Preconditioned polynomial (Algorithm A_p, preconditioning)."""

    def __init__(self, coeffs, p: int = 53, offset: int | None = None):
        self.coeffs = np.ascontiguousarray(np.asarray(coeffs, dtype=np.complex128))
        self._ri = self.coeffs.view(np.float64)
        self.p = int(p)
        self.d = self.coeffs.shape[0] - 1
        if offset is None:
            self._h = lib().ora_precondition(_ptr(self._ri, _f64p), self.d, self.p)
        else:   # threshold offset T given directly (worked example of Section 4.2)
            self._h = lib().ora_precondition_offset(_ptr(self._ri, _f64p), self.d, int(offset))
        if not self._h:
            raise MemoryError("oracle preconditioning failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().ora_plan_free(h)
            self._h = None

    def info(self) -> PlanInfo:
        o = np.zeros(7, np.int64)
        lib().ora_plan_info(self._h, _ptr(o, _i64p))
        return PlanInfo(*[int(x) for x in o])

    def hull(self):
        n = self.info().n_hull
        hk = np.zeros(max(n, 1), np.int64)
        hs = np.zeros(max(n, 1), np.int64)
        lib().ora_plan_hull(self._h, _ptr(hk, _i64p), _ptr(hs, _i64p))
        return hk[:n], hs[:n]

    def good(self) -> np.ndarray:
        g = np.zeros(self.d + 1, np.uint8)
        lib().ora_plan_good(self._h, _ptr(g, _u8p))
        return g.astype(bool)

    def scales(self) -> np.ndarray:
        s = np.zeros(self.d + 1, np.int64)
        lib().ora_plan_scales(self._h, _ptr(s, _i64p))
        return s

    def eval(self, z, nthreads: int | None = None) -> dict:
        """Q_lambda(z) per point, as (m, e) with Q = m 2^e, plus the plan quantities."""
        zri = _as_ri(np.atleast_1d(z))
        n = zri.shape[0] // 2
        m = np.zeros(2 * n, np.float64)
        e = np.zeros(n, np.int64)
        l = np.zeros(n, np.int64)
        r = np.zeros(n, np.int64)
        t = np.zeros(n, np.int64)
        dm = np.zeros(n, np.float64)
        de = np.zeros(n, np.int64)
        lam = np.zeros(n, np.float64)
        N = np.zeros(n, np.float64)
        lib().ora_eval(self._h, _ptr(zri, _f64p), n, _ptr(m, _f64p), _ptr(e, _i64p),
                       _ptr(l, _i64p), _ptr(r, _i64p), _ptr(t, _i64p), _ptr(dm, _f64p),
                       _ptr(de, _i64p), _ptr(lam, _f64p), _ptr(N, _f64p),
                       nthreads or default_threads())
        return {"m": m.view(np.complex128), "e": e, "l": l, "r": r, "terms": t,
                "dwin_m": dm, "dwin_e": de, "lambda": lam, "N": N}

    def eval_fp64(self, z, nthreads: int | None = None):
        """Q_lambda(z) with the window sum in plain FP64 (z^l by binary powering,
        Horner's rule over the window): (m, e) with Q = m 2^e."""
        zri = _as_ri(np.atleast_1d(z))
        n = zri.shape[0] // 2
        m = np.zeros(2 * n, np.float64)
        e = np.zeros(n, np.int64)
        lib().ora_eval_fp64(self._h, _ptr(zri, _f64p), n, _ptr(m, _f64p), _ptr(e, _i64p),
                            nthreads or default_threads())
        return m.view(np.complex128), e

    def level_sets(self, lam, dlevel=None):
        """N, x_L, x_R of eq. (def:LRN) at the given values of lambda (as eval
        computes them for a point with that lambda), the level moved to
        N - T + dlevel when dlevel is given."""
        lam = np.ascontiguousarray(np.atleast_1d(lam), np.float64)
        n = lam.shape[0]
        dl = None if dlevel is None else np.ascontiguousarray(np.broadcast_to(dlevel, (n,)), np.float64)
        N = np.zeros(n, np.float64)
        xl = np.zeros(n, np.float64)
        xr = np.zeros(n, np.float64)
        lib().ora_level_sets(self._h, _ptr(lam, _f64p), None if dl is None else _ptr(dl, _f64p), n, _ptr(N, _f64p), _ptr(xl, _f64p), _ptr(xr, _f64p))
        return N, xl, xr

    def cancel_bound(self, z, N, m, e) -> np.ndarray:
        """Upper bound of the cancelled bits c of eq. (def_prec_loss) per point,
        max(0, floor(N) + 1 - s(v)) for the value v = m 2^e (int32; 0 where the
        point has no window, INT32_MAX where v = 0); N as returned by eval."""
        zri = _as_ri(np.atleast_1d(z))
        n = zri.shape[0] // 2
        Nv = np.ascontiguousarray(np.asarray(N, np.float64).reshape(n))
        mri = _as_ri(np.atleast_1d(m))
        ev = np.ascontiguousarray(np.asarray(e, np.int64).reshape(n))
        out = np.zeros(n, np.int32)
        lib().ora_cancel_bound(self._h, _ptr(zri, _f64p), _ptr(Nv, _f64p), _ptr(mri, _f64p),
                               _ptr(ev, _i64p), n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        return out

    def eval_deriv(self, z, nthreads: int | None = None) -> dict:
        """Q_lambda(z) and Q'_lambda(z) = sum over the kept terms of k a_k z^(k-1),
        each as (m, e), with their window scales sum |a_k||z|^k and sum |k a_k||z|^(k-1)."""
        zri = _as_ri(np.atleast_1d(z))
        n = zri.shape[0] // 2
        m = np.zeros(2 * n, np.float64)
        e = np.zeros(n, np.int64)
        dm = np.zeros(n, np.float64)
        de = np.zeros(n, np.int64)
        md = np.zeros(2 * n, np.float64)
        ed = np.zeros(n, np.int64)
        ddm = np.zeros(n, np.float64)
        dde = np.zeros(n, np.int64)
        lib().ora_eval_deriv(self._h, _ptr(zri, _f64p), n, _ptr(m, _f64p), _ptr(e, _i64p), _ptr(dm, _f64p),
                             _ptr(de, _i64p), _ptr(md, _f64p), _ptr(ed, _i64p), _ptr(ddm, _f64p),
                             _ptr(dde, _i64p), nthreads or default_threads())
        return {"m": m.view(np.complex128), "e": e, "dwin_m": dm, "dwin_e": de,
                "md": md.view(np.complex128), "ed": ed, "ddwin_m": ddm, "ddwin_e": dde}


    def adjoint(self, z, g) -> dict:
        """Reverse mode of Q_lambda at the points z for upstream gradients g, in the
        convention of complex reverse mode (upstream gradient times the conjugate
        derivative), the kept set held fixed:
          grad_a[k] = sum over the points keeping k of g_j conj(z_j)^k   (as ga_m 2^ga_e,
                      with its scale sum |g_j| |z_j|^k as ga_scale_m 2^ga_scale_e),
          grad_z[j] = g_j conj(Q'_lambda(z_j))                            (as gz_m 2^gz_e,
                      with its scale |g_j| sum |k a_k||z_j|^(k-1) as gz_scale_m 2^gz_scale_e).
        """
        zri = _as_ri(np.atleast_1d(z))
        gri = _as_ri(np.atleast_1d(g))
        n = zri.shape[0] // 2
        if gri.shape[0] != 2 * n:
            raise ValueError("z and g differ in length")
        ga = np.zeros(2 * (self.d + 1), np.float64)
        gae = np.zeros(self.d + 1, np.int64)
        sm = np.zeros(self.d + 1, np.float64)
        se = np.zeros(self.d + 1, np.int64)
        lib().ora_adjoint_coef(self._h, _ptr(zri, _f64p), _ptr(gri, _f64p), n, self.d, _ptr(ga, _f64p),
                               _ptr(gae, _i64p), _ptr(sm, _f64p), _ptr(se, _i64p))
        dv = self.eval_deriv(zri.view(np.complex128))
        gc = gri.view(np.complex128)
        return {"ga_m": ga.view(np.complex128), "ga_e": gae, "ga_scale_m": sm, "ga_scale_e": se,
                "gz_m": gc * np.conj(dv["md"]), "gz_e": dv["ed"],
                "gz_scale_m": np.abs(gc) * dv["ddwin_m"], "gz_scale_e": dv["ddwin_e"]}

def precondition(coeffs, p: int = 53, offset: int | None = None) -> OraclePlan:
    return OraclePlan(coeffs, p, offset)


def horner(coeffs, z, nthreads: int | None = None):
    """P(z) for the full polynomial by compensated Horner; returns (m, e), P = m 2^e."""
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.complex128))
    cri = c.view(np.float64)
    zri = _as_ri(np.atleast_1d(z))
    n = zri.shape[0] // 2
    m = np.zeros(2 * n, np.float64)
    e = np.zeros(n, np.int64)
    lib().ora_horner(_ptr(cri, _f64p), c.shape[0] - 1, _ptr(zri, _f64p), n,
                     _ptr(m, _f64p), _ptr(e, _i64p), nthreads or default_threads())
    return m.view(np.complex128), e


def absum(coeffs, z, nthreads: int | None = None):
    """D(z) = sum_k |a_k| |z|^k; returns (m, e), D = m 2^e."""
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.complex128))
    cri = c.view(np.float64)
    zri = _as_ri(np.atleast_1d(z))
    n = zri.shape[0] // 2
    m = np.zeros(n, np.float64)
    e = np.zeros(n, np.int64)
    lib().ora_absum(_ptr(cri, _f64p), c.shape[0] - 1, _ptr(zri, _f64p), n,
                    _ptr(m, _f64p), _ptr(e, _i64p), nthreads or default_threads())
    return m, e


def scaled_error(m_a, e_a, m_b, e_b, d_m, d_e) -> np.ndarray:
    """|A - B| / D for numbers given as mantissa 2^exponent (no overflow).

    Each operand is rebased to D's exponent before the subtraction.  This is the
    parity metric: max over points of |FPE - reference| / sum_k |a_k||z|^k.
    """
    m_a = np.asarray(m_a, np.complex128)
    m_b = np.asarray(m_b, np.complex128)
    d_m = np.asarray(d_m, np.float64)
    sa = np.clip(np.asarray(e_a, np.int64) - np.asarray(d_e, np.int64), -3000, 3000)
    sb = np.clip(np.asarray(e_b, np.int64) - np.asarray(d_e, np.int64), -3000, 3000)
    with np.errstate(over="ignore", invalid="ignore"):
        a = np.ldexp(m_a.real, sa) + 1j * np.ldexp(m_a.imag, sa)
        b = np.ldexp(m_b.real, sb) + 1j * np.ldexp(m_b.imag, sb)
        err = np.abs(a - b) / d_m
    zero = (d_m == 0) & (np.abs(m_a) == 0) & (np.abs(m_b) == 0)
    err[zero] = 0.0
    return err
