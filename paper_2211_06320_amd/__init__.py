"""Python binding of libfpe, the MI355X Fast Polynomial Evaluator (arXiv 2211.06320).

Thin ctypes marshalling over the C ABI declared in include/fpe.h: every step of
preconditioning and evaluation runs in the HIP library; PyTorch provides device
memory (all buffers, including workspaces, are torch tensors) and the stream.
There is no fallback: if libfpe.so is missing, loading fails with an error.

    plan = precondition(coeffs)            # coeffs: complex128 CUDA tensor, a_0 first
    plan32 = precondition(coeffs, 24, fp32=True)   # FP32 window sums at p = 24
    m, e = plan.eval(z)                    # P(z) ~ m * 2**e, m complex128, e int64
    m, e, terms, window = plan.eval(z, terms=True, window=True)
    m, e = horner_eval(coeffs, z)          # same-GPU Horner baseline
    to_complex(m, e)                       # m * 2**e as complex128 (may overflow)
    m, e, md, ed = plan.eval_deriv(z)      # and Q' = md * 2**ed through the same window
    ga, gz = plan.adjoint(z, g)            # reverse mode for upstream gradients g
    q = fpe_eval(coeffs, z)                # differentiable (torch.autograd)
    q, e = eval_scaled(plan, coeffs, z)    # differentiable normalised values, Q = q 2^e
    cov = Cover(coeffs); p53, p24 = cov.plan(53), cov.plan(24)    # the cover once, G_p per precision
    plans = precondition_batched([c1, c2, c3])                      # many polynomials, one launch sequence
    b = Batch([plan_a, plan_b], [0, na, na + nb]); m, e = b.eval(z_ab)   # many polynomials at once
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfpe.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "fpe.h")

FPE_OK = 0
PRECONDITION_FP32 = 1
PRECONDITION_FP32_COMPENSATED = 2
WINDOW_AUTO, WINDOW_DENSE, WINDOW_SPARSE = 0, 1, 2
ADJOINT_EXACT, ADJOINT_ATOMIC = 0, 1
STATUS = {0: "FPE_OK", 1: "FPE_ERR_INVALID_ARG", 2: "FPE_ERR_NONFINITE", 3: "FPE_ERR_PRECISION",
          4: "FPE_ERR_WORKSPACE", 5: "FPE_ERR_HIP", 6: "FPE_ERR_UNSUPPORTED"}

_LIB = None


class FPEError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {detail}")


def header_functions() -> list[str]:
    """Names of the functions declared in include/fpe.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fpe_[a-z_0-9]+)\s*\(", txt)))


def lib() -> ctypes.CDLL:
    """Load libfpe.so (built by __graft_entry__.build()); raises if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
    P = ctypes.POINTER
    L.fpe_status_string.restype = ctypes.c_char_p
    L.fpe_status_string.argtypes = [i32]
    L.fpe_last_error.restype = ctypes.c_char_p
    L.fpe_last_error.argtypes = []
    L.fpe_abi_version.restype = i32
    L.fpe_precondition_workspace_size.restype = i32
    L.fpe_precondition_workspace_size.argtypes = [i64, i32, u32, P(sz)]
    L.fpe_precondition.restype = i32
    L.fpe_precondition.argtypes = [vp, i64, i32, u32, vp, sz, vp, P(vp)]
    L.fpe_cover_workspace_size.restype = i32
    L.fpe_cover_workspace_size.argtypes = [i64, P(sz)]
    L.fpe_cover_build.restype = i32
    L.fpe_cover_build.argtypes = [vp, i64, vp, sz, vp, P(vp)]
    L.fpe_cover_info.restype = i32
    L.fpe_cover_info.argtypes = [vp, P(i64)]
    L.fpe_cover_destroy.restype = i32
    L.fpe_cover_destroy.argtypes = [vp]
    L.fpe_plan_from_cover_workspace_size.restype = i32
    L.fpe_plan_from_cover_workspace_size.argtypes = [vp, i32, u32, P(sz)]
    L.fpe_plan_from_cover.restype = i32
    L.fpe_plan_from_cover.argtypes = [vp, vp, i32, u32, vp, sz, vp, P(vp)]
    L.fpe_precondition_batched_workspace_size.restype = i32
    L.fpe_precondition_batched_workspace_size.argtypes = [i32, P(i64), i32, u32, P(sz)]
    L.fpe_precondition_batched.restype = i32
    L.fpe_precondition_batched.argtypes = [vp, P(i64), i32, i32, u32, vp, sz, vp, P(vp)]
    L.fpe_plan_info.restype = i32
    L.fpe_plan_info.argtypes = [vp, P(i64)]
    L.fpe_plan_export.restype = i32
    L.fpe_plan_export.argtypes = [vp, P(i64), P(i64), i64, P(ctypes.c_uint8)]
    L.fpe_plan_destroy.restype = i32
    L.fpe_plan_destroy.argtypes = [vp]
    L.fpe_eval_workspace_size.restype = i32
    L.fpe_eval_workspace_size.argtypes = [vp, i64, P(sz)]
    L.fpe_eval.restype = i32
    L.fpe_eval.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, sz, vp]
    L.fpe_eval_noalloc.restype = i32
    L.fpe_eval_noalloc.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
    L.fpe_eval_deriv.restype = i32
    L.fpe_eval_deriv.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, sz, vp]
    L.fpe_newton_step.restype = i32
    L.fpe_newton_step.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, sz, vp]
    L.fpe_batch_workspace_size.restype = i32
    L.fpe_batch_workspace_size.argtypes = [i32, P(i64), P(sz)]
    L.fpe_batch_create.restype = i32
    L.fpe_batch_create.argtypes = [P(vp), i32, P(i64), vp, sz, vp, P(vp)]
    L.fpe_batch_destroy.restype = i32
    L.fpe_batch_destroy.argtypes = [vp]
    L.fpe_eval_batched_workspace_size.restype = i32
    L.fpe_eval_batched_workspace_size.argtypes = [vp, P(sz)]
    L.fpe_eval_batched.restype = i32
    L.fpe_eval_batched.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    L.fpe_plan_set_chunk.restype = i32
    L.fpe_plan_set_chunk.argtypes = [vp, i32]
    L.fpe_plan_set_window_mode.restype = i32
    L.fpe_plan_set_window_mode.argtypes = [vp, i32]
    L.fpe_plan_set_adjoint_mode.restype = i32
    L.fpe_plan_set_adjoint_mode.argtypes = [vp, i32]
    L.fpe_plan_tile_choice.restype = i32
    L.fpe_plan_tile_choice.argtypes = [vp, i64, P(i32), P(i32)]
    L.fpe_autotune.restype = i32
    L.fpe_autotune.argtypes = [vp, vp, i64, vp, vp, vp, sz, vp, P(i32)]
    L.fpe_batch_set_chunk.restype = i32
    L.fpe_batch_set_chunk.argtypes = [vp, i32]
    L.fpe_batch_autotune.restype = i32
    L.fpe_batch_autotune.argtypes = [vp, vp, vp, vp, vp, sz, vp, P(i32)]
    L.fpe_eval_adjoint.restype = i32
    L.fpe_eval_adjoint.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.fpe_cancelled_bits.restype = i32
    L.fpe_cancelled_bits.argtypes = [vp, vp, i64, vp, vp, vp, vp]
    L.fpe_horner_eval.restype = i32
    L.fpe_horner_eval.argtypes = [vp, i64, vp, i64, vp, vp, vp]
    L.fpe_profile_enable.restype = i32
    L.fpe_profile_enable.argtypes = [i32]
    L.fpe_profile_read.restype = i32
    L.fpe_profile_read.argtypes = [P(ctypes.c_double), P(i64)]
    _LIB = L
    return L


def _check(status: int):
    if status != FPE_OK:
        raise FPEError(status, lib().fpe_last_error().decode())


def _torch():
    import torch
    return torch


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _flags(fp32: bool, compensated: bool) -> int:
    if compensated and not fp32:
        raise ValueError("compensated FP32 blocks need fp32=True")
    return (PRECONDITION_FP32 if fp32 else 0) | (PRECONDITION_FP32_COMPENSATED if compensated else 0)


def _dev_complex(x, name):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or x.dtype != torch.complex128 or not x.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    return x.contiguous()


def _workspace(nbytes: int, device):
    """Caller-owned device workspace (torch memory), 256-byte aligned."""
    torch = _torch()
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


@dataclass
class PlanInfo:
    d: int
    v: int
    dt: int
    n_hull: int
    n_good: int
    T: int
    p: int
    chunk: int
    s_max: int
    s_min_good: int


class Plan:
    """A polynomial preconditioned by fpe_precondition (Algorithm A_p, first block)."""

    def __init__(self, coeffs, p: int = 53, stream=None, fp32: bool = False, compensated: bool = False):
        L = lib()
        coeffs = _dev_complex(coeffs, "coeffs")
        d = coeffs.shape[0] - 1
        flags = _flags(fp32, compensated)
        nb = ctypes.c_size_t()
        _check(L.fpe_precondition_workspace_size(d, p, flags, ctypes.byref(nb)))
        ws_buf, ws = _workspace(nb.value, coeffs.device)
        h = ctypes.c_void_p()
        _check(L.fpe_precondition(coeffs.data_ptr(), d, p, flags, ws, nb.value,
                                  _stream(stream), ctypes.byref(h)))
        self._adopt(h, ws_buf, coeffs.device, d, fp32)

    def _adopt(self, h, ws_buf, device, d: int, fp32: bool):
        self._h = h
        self._ws_buf = ws_buf                  # the plan's tables live here
        self.device = device
        self.d = int(d)
        self.fp32 = bool(fp32)
        self._eval_ws = {}
        self._destroy = lib().fpe_plan_destroy     # kept: module globals may be gone at exit

    @classmethod
    def _from_handle(cls, h, ws_buf, device, d: int, fp32: bool):
        obj = cls.__new__(cls)
        obj._adopt(h, ws_buf, device, d, fp32)
        return obj

    def __del__(self):
        h = getattr(self, "_h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self._h = None

    def info(self) -> PlanInfo:
        import numpy as np
        out = np.zeros(10, np.int64)
        _check(lib().fpe_plan_info(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return PlanInfo(*[int(x) for x in out])

    def export(self):
        """(hull_k, hull_s, good) as numpy arrays."""
        import numpy as np
        nh = self.info().n_hull
        hk = np.zeros(max(nh, 1), np.int64)
        hs = np.zeros(max(nh, 1), np.int64)
        good = np.zeros(self.d + 1, np.uint8)
        i64p = ctypes.POINTER(ctypes.c_int64)
        _check(lib().fpe_plan_export(self._h, hk.ctypes.data_as(i64p), hs.ctypes.data_as(i64p), max(nh, 1),
                                     good.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
        return hk[:nh], hs[:nh], good.astype(bool)

    def eval_workspace_bytes(self, n: int) -> int:
        nb = ctypes.c_size_t()
        _check(lib().fpe_eval_workspace_size(self._h, n, ctypes.byref(nb)))
        return nb.value

    def workspace(self, n: int, stream=None):
        """A cached device workspace large enough for n points, one per stream:
        calls on different streams may overlap, so they never share one."""
        torch = _torch()
        nb = self.eval_workspace_bytes(n)
        s = stream if stream is not None else torch.cuda.current_stream()
        key = int(s.cuda_stream)
        cur = self._eval_ws.get(key)
        if cur is None or cur[2] < nb:
            buf, ptr = _workspace(nb, self.device)
            # the caching allocator may hand the memory out again only once the
            # work queued on this stream is done with it
            if s != torch.cuda.current_stream():
                buf.record_stream(s)
            self._eval_ws[key] = (buf, ptr, nb)
        return self._eval_ws[key][1], self._eval_ws[key][2]

    def eval(self, z, terms: bool = False, window: bool = False, out=None, stream=None):
        """Q_lambda(z) for every point (Algorithm A_p, second block).

        Returns (m, e) or (m, e, terms, window): m complex128 [n], e int64 [n],
        terms int32 [n] (#G_p within [l, r]), window int64 [n, 2] ((l, r)).
        """
        torch = _torch()
        z = _dev_complex(z, "z")
        n = z.shape[0]
        if out is None:
            m = torch.empty(n, dtype=torch.complex128, device=z.device)
            e = torch.empty(n, dtype=torch.int64, device=z.device)
        else:
            m, e = out
        t = torch.empty(n, dtype=torch.int32, device=z.device) if terms else None
        w = torch.empty((n, 2), dtype=torch.int64, device=z.device) if window else None
        ws, nb = self.workspace(n, stream)
        _check(lib().fpe_eval(self._h, z.data_ptr(), n, m.data_ptr(), e.data_ptr(),
                              t.data_ptr() if t is not None else None,
                              w.data_ptr() if w is not None else None, ws, nb, _stream(stream)))
        if terms or window:
            return m, e, t, w
        return m, e


    def eval_noalloc(self, z, out, terms=None, window=None, stream=None):
        """fpe_eval_noalloc: Q_lambda(z) into the caller's tensors out = (m, e)
        (and terms / window when given), with the library's static device
        scratch as workspace; allocates nothing."""
        z = _dev_complex(z, "z")
        m, e = out
        _check(lib().fpe_eval_noalloc(self._h, z.data_ptr(), z.shape[0], m.data_ptr(), e.data_ptr(),
                                      terms.data_ptr() if terms is not None else None,
                                      window.data_ptr() if window is not None else None, _stream(stream)))
        return m, e

    def set_chunk(self, chunk: int) -> None:
        """Chunk length of the tiles for later evaluations (0: automatic)."""
        _check(lib().fpe_plan_set_chunk(self._h, int(chunk)))

    def set_window_mode(self, mode) -> None:
        """Window-sum form of later evaluations: "auto", "dense" or "sparse"
        (or WINDOW_AUTO / WINDOW_DENSE / WINDOW_SPARSE)."""
        m = {"auto": WINDOW_AUTO, "dense": WINDOW_DENSE, "sparse": WINDOW_SPARSE}.get(mode, mode)
        _check(lib().fpe_plan_set_window_mode(self._h, int(m)))

    def set_adjoint_mode(self, mode) -> None:
        """How adjoint sums grad_a: "exact" (fixed point, the same bits every
        call; the default) or "atomic" (FP64 atomics, faster)."""
        m = {"exact": ADJOINT_EXACT, "atomic": ADJOINT_ATOMIC}.get(mode, mode)
        _check(lib().fpe_plan_set_adjoint_mode(self._h, int(m)))

    def tile_choice(self, n: int):
        """(chunk length, "dense" or "sparse") an evaluation of n points would use."""
        c, m = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fpe_plan_tile_choice(self._h, int(n), ctypes.byref(c), ctypes.byref(m)))
        return c.value, ("sparse" if m.value == WINDOW_SPARSE else "dense")

    def autotune(self, z, stream=None) -> int:
        """Times the candidate chunk lengths and window-sum forms on these
        points, keeps the fastest pair; returns the chunk length."""
        torch = _torch()
        z = _dev_complex(z, "z")
        n = z.shape[0]
        m = torch.empty(n, dtype=torch.complex128, device=z.device)
        e = torch.empty(n, dtype=torch.int64, device=z.device)
        ws, nb = self.workspace(n, stream)
        c = ctypes.c_int32()
        _check(lib().fpe_autotune(self._h, z.data_ptr(), n, m.data_ptr(), e.data_ptr(), ws, nb, _stream(stream),
                                  ctypes.byref(c)))
        return c.value

    def eval_deriv(self, z, stream=None):
        """Q_lambda(z) and its derivative through the same window; returns
        (m, e, md, ed) with Q = m 2^e and Q' = md 2^ed."""
        torch = _torch()
        z = _dev_complex(z, "z")
        n = z.shape[0]
        m = torch.empty(n, dtype=torch.complex128, device=z.device)
        e = torch.empty(n, dtype=torch.int64, device=z.device)
        md = torch.empty(n, dtype=torch.complex128, device=z.device)
        ed = torch.empty(n, dtype=torch.int64, device=z.device)
        ws, nb = self.workspace(n, stream)
        _check(lib().fpe_eval_deriv(self._h, z.data_ptr(), n, m.data_ptr(), e.data_ptr(), md.data_ptr(),
                                    ed.data_ptr(), ws, nb, _stream(stream)))
        return m, e, md, ed

    def newton_step(self, z, stream=None):
        """One Newton step z - Q/Q' per point; returns (z_new, m, e, md, ed)."""
        torch = _torch()
        z = _dev_complex(z, "z")
        n = z.shape[0]
        m = torch.empty(n, dtype=torch.complex128, device=z.device)
        e = torch.empty(n, dtype=torch.int64, device=z.device)
        md = torch.empty(n, dtype=torch.complex128, device=z.device)
        ed = torch.empty(n, dtype=torch.int64, device=z.device)
        zn = torch.empty(n, dtype=torch.complex128, device=z.device)
        ws, nb = self.workspace(n, stream)
        _check(lib().fpe_newton_step(self._h, z.data_ptr(), n, m.data_ptr(), e.data_ptr(), md.data_ptr(),
                                     ed.data_ptr(), zn.data_ptr(), ws, nb, _stream(stream)))
        return zn, m, e, md, ed

    def cancelled_bits(self, z, m=None, e=None, stream=None):
        """Upper bound of the cancelled bits c of eq. (def_prec_loss) per point for
        the values m 2^e (this plan's eval of z when not given): int32 tensor,
        max(0, floor(N) + 1 - s(m 2^e)); at least p - bits - 2 leading bits of
        the value are correct."""
        torch = _torch()
        z = _dev_complex(z, "z")
        if m is None or e is None:
            m, e = self.eval(z, stream=stream)
        m = _dev_complex(m, "m")
        if m.shape != z.shape or e.shape != z.shape or e.dtype != torch.int64 or e.device != z.device:
            raise ValueError("m and e must be [n] complex128 and int64 on the device of z")
        e = e.contiguous()
        bits = torch.empty(z.shape[0], dtype=torch.int32, device=z.device)
        _check(lib().fpe_cancelled_bits(self._h, z.data_ptr(), z.shape[0], m.data_ptr(), e.data_ptr(),
                                        bits.data_ptr(), _stream(stream)))
        return bits

    def adjoint(self, z, g, md=None, ed=None, grad_a: bool = True, grad_z: bool = True, g_exp=None, stream=None):
        """Reverse mode of Q_lambda for upstream gradients g (complex convention:
        upstream gradient times the conjugate derivative; the kept terms held
        fixed).  Returns (grad_a [d + 1] or None, grad_z [n] or None):
        grad_a[k] = sum of g_j conj(z_j)^k over the points keeping k,
        grad_z[j] = g_j conj(Q'(z_j)), Q' = md 2^ed from eval_deriv (computed
        here when not given).  g_exp (int64 [n], optional): the upstream
        gradients are g_j 2^(-g_exp[j])."""
        torch = _torch()
        z = _dev_complex(z, "z")
        g = _dev_complex(g, "g")
        n = z.shape[0]
        if g.shape != z.shape:
            raise ValueError("g must have the shape of z")
        if g_exp is not None:
            if g_exp.shape != z.shape or g_exp.dtype != torch.int64 or g_exp.device != z.device:
                raise ValueError("g_exp must be an int64 tensor shaped like z on its device")
            g_exp = g_exp.contiguous()
        if grad_z and (md is None or ed is None):
            _, _, md, ed = self.eval_deriv(z, stream=stream)
        ga = torch.empty(self.d + 1, dtype=torch.complex128, device=z.device) if grad_a else None
        gz = torch.empty(n, dtype=torch.complex128, device=z.device) if grad_z else None
        if grad_z:
            md = _dev_complex(md, "md")
            ed = ed.contiguous()
        ws, nb = self.workspace(n, stream)
        _check(lib().fpe_eval_adjoint(self._h, z.data_ptr(), n, g.data_ptr(),
                                      g_exp.data_ptr() if g_exp is not None else None,
                                      md.data_ptr() if grad_z else None, ed.data_ptr() if grad_z else None,
                                      ga.data_ptr() if ga is not None else None,
                                      gz.data_ptr() if gz is not None else None, ws, nb, _stream(stream)))
        return ga, gz


class Batch:
    """Many polynomials, each with its own points, evaluated by one launch
    sequence (fpe_eval_batched).  plans: Plan objects (kept alive by the batch);
    offsets: n_poly + 1 integers, polynomial i owns points offsets[i] ..
    offsets[i+1] - 1 of the concatenated point array."""

    def __init__(self, plans, offsets, stream=None):
        L = lib()
        self.plans = list(plans)
        offs = [int(x) for x in offsets]
        n_poly = len(self.plans)
        if len(offs) != n_poly + 1:
            raise ValueError("offsets must have len(plans) + 1 entries")
        self.n_points = offs[-1]
        self.device = self.plans[0].device
        c_offs = (ctypes.c_int64 * len(offs))(*offs)
        nb = ctypes.c_size_t()
        _check(L.fpe_batch_workspace_size(n_poly, c_offs, ctypes.byref(nb)))
        self._ws_buf, ws = _workspace(nb.value, self.device)
        handles = (ctypes.c_void_p * n_poly)(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(L.fpe_batch_create(handles, n_poly, c_offs, ws, nb.value, _stream(stream), ctypes.byref(h)))
        self._h = h
        self._destroy = L.fpe_batch_destroy
        enb = ctypes.c_size_t()
        _check(L.fpe_eval_batched_workspace_size(h, ctypes.byref(enb)))
        self._eval_nb = enb.value
        self._eval_ws = {}
        self.eval_workspace(stream)

    def eval_workspace(self, stream=None) -> int:
        """The evaluation workspace for calls on this stream (one per stream:
        calls on different streams may overlap)."""
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream()
        key = int(s.cuda_stream)
        if key not in self._eval_ws:
            buf, ptr = _workspace(self._eval_nb, self.device)
            if s != torch.cuda.current_stream():
                buf.record_stream(s)
            self._eval_ws[key] = (buf, ptr)
        return self._eval_ws[key][1]

    def __del__(self):
        h = getattr(self, "_h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self._h = None

    def set_chunk(self, chunk: int) -> None:
        """Chunk length of the tiles for later evaluations (0: automatic)."""
        _check(lib().fpe_batch_set_chunk(self._h, int(chunk)))

    def autotune(self, z, stream=None) -> int:
        """Times the candidate chunk lengths on these points, keeps the fastest."""
        torch = _torch()
        z = _dev_complex(z, "z")
        n = self.n_points
        m = torch.empty(n, dtype=torch.complex128, device=z.device)
        e = torch.empty(n, dtype=torch.int64, device=z.device)
        c = ctypes.c_int32()
        _check(lib().fpe_batch_autotune(self._h, z.data_ptr(), m.data_ptr(), e.data_ptr(),
                                        self.eval_workspace(stream), self._eval_nb, _stream(stream),
                                        ctypes.byref(c)))
        return c.value

    def eval(self, z, terms: bool = False, out=None, stream=None):
        """Q_lambda at every point of every polynomial: (m, e) or (m, e, terms)."""
        torch = _torch()
        z = _dev_complex(z, "z")
        if z.shape[0] != self.n_points:
            raise ValueError(f"expected {self.n_points} points")
        n = self.n_points
        if out is None:
            m = torch.empty(n, dtype=torch.complex128, device=z.device)
            e = torch.empty(n, dtype=torch.int64, device=z.device)
        else:
            m, e = out
        t = torch.empty(n, dtype=torch.int32, device=z.device) if terms else None
        _check(lib().fpe_eval_batched(self._h, z.data_ptr(), m.data_ptr(), e.data_ptr(),
                                      t.data_ptr() if t is not None else None, self.eval_workspace(stream),
                                      self._eval_nb, _stream(stream)))
        return (m, e, t) if terms else (m, e)


def _fpe_function():
    torch = _torch()

    class FPEEval(torch.autograd.Function):
        """Q_lambda(z) as complex128 for coefficients a (precondition + eval), with
        the backward pass of fpe_eval_adjoint.  The map is piecewise polynomial:
        the kept set (G_p and the windows) is held fixed under differentiation."""

        @staticmethod
        def forward(ctx, coeffs, z, p):
            plan = Plan(coeffs.detach(), p)
            zd = z.detach()
            if ctx.needs_input_grad[1]:
                m, e, md, ed = plan.eval_deriv(zd)
            else:
                m, e = plan.eval(zd)
                md = ed = None
            ctx.plan = plan
            ctx.z, ctx.md, ctx.ed = zd, md, ed
            return to_complex(m, e)

        @staticmethod
        def backward(ctx, g):
            ga, gz = ctx.plan.adjoint(ctx.z, g.contiguous(), ctx.md, ctx.ed,
                                      grad_a=ctx.needs_input_grad[0], grad_z=ctx.needs_input_grad[1])
            return ga, gz, None

    return FPEEval


def _fpe_scaled_function():
    torch = _torch()

    class FPEEvalScaled(torch.autograd.Function):
        """Q_lambda(z) = q 2^e per point for a prebuilt plan of the coefficients a:
        q complex128 (normalised mantissas, differentiable) and e int64 (the
        binary exponents, treated as constants).  The backward pass is
        fpe_eval_adjoint with the upstream gradient of q passed as g 2^-e, so a
        loss on the normalised values (say sum |q_j|^2 = sum |Q_j|^2 4^-e_j)
        backpropagates without any value leaving the double range.  The plan
        must have been preconditioned from a (its kept set is held fixed)."""

        @staticmethod
        def forward(ctx, coeffs, z, plan):
            zd = z.detach()
            if ctx.needs_input_grad[1]:
                m, e, md, ed = plan.eval_deriv(zd)
            else:
                m, e = plan.eval(zd)
                md = ed = None
            ctx.plan = plan
            ctx.z, ctx.e, ctx.md, ctx.ed = zd, e, md, ed
            ctx.mark_non_differentiable(e)
            return m, e

        @staticmethod
        def backward(ctx, gq, ge):
            if gq is None:
                return None, None, None
            ga, gz = ctx.plan.adjoint(ctx.z, gq.contiguous(), ctx.md, ctx.ed, grad_a=ctx.needs_input_grad[0],
                                      grad_z=ctx.needs_input_grad[1], g_exp=ctx.e)
            return ga, gz, None

    return FPEEvalScaled


_FPE_FN = None
_FPE_SCALED_FN = None


def fpe_eval(coeffs, z, p: int = 53):
    """Differentiable Q_lambda(z) (complex128, may overflow to inf like to_complex)."""
    global _FPE_FN
    if _FPE_FN is None:
        _FPE_FN = _fpe_function()
    return _FPE_FN.apply(_dev_complex(coeffs, "coeffs"), _dev_complex(z, "z"), p)


def eval_scaled(plan, coeffs, z):
    """Differentiable (q, e) with Q_lambda(z_j) = q_j 2^(e_j) for a prebuilt plan
    of coeffs: q complex128 [n] differentiable in coeffs and z, e int64 [n]
    constant.  Losses on q stay in range where |Q| itself leaves the double range."""
    global _FPE_SCALED_FN
    if _FPE_SCALED_FN is None:
        _FPE_SCALED_FN = _fpe_scaled_function()
    return _FPE_SCALED_FN.apply(_dev_complex(coeffs, "coeffs"), _dev_complex(z, "z"), plan)


class Cover:
    """The scales and the concave cover of a polynomial (fpe_cover_build), which
    do not depend on p; plan(p) finishes the preconditioning for a precision
    (fpe_plan_from_cover: G_p and the tables), as often as needed."""

    def __init__(self, coeffs, stream=None):
        L = lib()
        self.coeffs = _dev_complex(coeffs, "coeffs")     # kept: plan() reads them again
        self.device = self.coeffs.device
        self.d = self.coeffs.shape[0] - 1
        nb = ctypes.c_size_t()
        _check(L.fpe_cover_workspace_size(self.d, ctypes.byref(nb)))
        self._ws_buf, ws = _workspace(nb.value, self.device)
        h = ctypes.c_void_p()
        _check(L.fpe_cover_build(self.coeffs.data_ptr(), self.d, ws, nb.value, _stream(stream), ctypes.byref(h)))
        self._h = h
        self._destroy = L.fpe_cover_destroy

    def __del__(self):
        h = getattr(self, "_h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self._h = None

    def info(self):
        """(d, v, d', number of cover vertices, max s(a_k))."""
        import numpy as np
        out = np.zeros(5, np.int64)
        _check(lib().fpe_cover_info(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return tuple(int(x) for x in out)

    def plan(self, p: int = 53, fp32: bool = False, stream=None, compensated: bool = False) -> Plan:
        L = lib()
        flags = _flags(fp32, compensated)
        nb = ctypes.c_size_t()
        _check(L.fpe_plan_from_cover_workspace_size(self._h, p, flags, ctypes.byref(nb)))
        ws_buf, ws = _workspace(nb.value, self.device)
        h = ctypes.c_void_p()
        _check(L.fpe_plan_from_cover(self._h, self.coeffs.data_ptr(), p, flags, ws, nb.value, _stream(stream),
                                     ctypes.byref(h)))
        return Plan._from_handle(h, ws_buf, self.device, self.d, fp32)


def precondition_batched(coeffs, p: int = 53, fp32: bool = False, stream=None, compensated: bool = False) -> list:
    """Plans for many polynomials from one launch sequence (fpe_precondition_batched).
    coeffs: a list of complex128 CUDA tensors (a_0 first each).  The plans share
    one workspace (held by each of them)."""
    torch = _torch()
    L = lib()
    parts = [_dev_complex(c, "coeffs") for c in coeffs]
    if not parts:
        return []
    flat = torch.cat(parts)
    offs = [0]
    for c in parts:
        offs.append(offs[-1] + int(c.shape[0]))
    n_poly = len(parts)
    c_offs = (ctypes.c_int64 * len(offs))(*offs)
    flags = _flags(fp32, compensated)
    nb = ctypes.c_size_t()
    _check(L.fpe_precondition_batched_workspace_size(n_poly, c_offs, p, flags, ctypes.byref(nb)))
    ws_buf, ws = _workspace(nb.value, flat.device)
    handles = (ctypes.c_void_p * n_poly)()
    _check(L.fpe_precondition_batched(flat.data_ptr(), c_offs, n_poly, p, flags, ws, nb.value, _stream(stream),
                                      handles))
    return [Plan._from_handle(ctypes.c_void_p(handles[i]), ws_buf, flat.device, offs[i + 1] - offs[i] - 1, fp32)
            for i in range(n_poly)]


def precondition(coeffs, p: int = 53, stream=None, fp32: bool = False, compensated: bool = False) -> Plan:
    """fp32=True (p <= 24): fpe_eval sums the windows in FP32 (FPE_PRECONDITION_FP32);
    compensated=True with it: the FP32 blocks by the compensated (TwoSum/TwoProd)
    recurrence (FPE_PRECONDITION_FP32_COMPENSATED)."""
    return Plan(coeffs, p, stream, fp32, compensated)


def horner_eval(coeffs, z, out=None, stream=None):
    """P(z) for the full polynomial by Horner's rule on the GPU; returns (m, e)."""
    torch = _torch()
    coeffs = _dev_complex(coeffs, "coeffs")
    z = _dev_complex(z, "z")
    n = z.shape[0]
    if out is None:
        m = torch.empty(n, dtype=torch.complex128, device=z.device)
        e = torch.empty(n, dtype=torch.int64, device=z.device)
    else:
        m, e = out
    _check(lib().fpe_horner_eval(coeffs.data_ptr(), coeffs.shape[0] - 1, z.data_ptr(), n,
                                 m.data_ptr(), e.data_ptr(), _stream(stream)))
    return m, e


def profile_enable(on: bool = True) -> None:
    """Record HIP events around every later window-kernel launch (measurement only)."""
    _check(lib().fpe_profile_enable(1 if on else 0))


def profile_read():
    """(summed window-kernel milliseconds, launches) since the last read."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().fpe_profile_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def to_complex(m, e):
    """m * 2**e as complex128 (overflows to inf where the value leaves the FP64 range)."""
    torch = _torch()
    ee = e.clamp(-3000, 3000).to(torch.float64)
    sc = torch.pow(2.0, ee)
    return torch.complex(m.real * sc, m.imag * sc)
