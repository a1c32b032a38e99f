"""Host build of the kernels' double-double powering, checked against mpmath."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def hm(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    so = str(tmp_path_factory.mktemp("hm") / "host_math.so")
    # -mfma -ffp-contract=fast: contraction would happen here too if a helper allowed it
    subprocess.run([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                    "-mfma", "-ffp-contract=fast",
                    "-Wno-unused-command-line-argument", "-o", so, os.path.join(HERE, "host_math.cpp")],
                   check=True, capture_output=True)
    L = ctypes.CDLL(so)
    dp = ctypes.POINTER(ctypes.c_double)
    L.hm_cdd_sqr.argtypes = [dp, dp]
    L.hm_cdd_mul_d.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
    L.hm_chunk_start.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                 dp, dp, ctypes.POINTER(ctypes.c_longlong)]
    L.hm_cdd_renorm.argtypes = [dp, dp, ctypes.POINTER(ctypes.c_longlong)]
    L.hm_cpow.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int,
                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(ctypes.c_longlong)]
    return L


def test_cpow_dd_against_mpmath(hm):
    """w^n with w normalised (max component in [1/2, 1)): relative error <= 2^-52
    after rounding (each component rounded once; the double-double part stays
    below 2^-62 for any int exponent)."""
    import mpmath
    mpmath.mp.prec = 256
    rng = np.random.default_rng(4)
    pr, pi, E = ctypes.c_double(), ctypes.c_double(), ctypes.c_longlong()
    ns = [0, 1, 2, 3, 7, 64, 952, 1000, 4095, 999_999, 1 << 20, (1 << 30) + 12345, (1 << 31) - 1]
    for _ in range(200):
        t = rng.uniform(0, 2 * np.pi)
        w = complex(np.cos(t), np.sin(t)) * rng.uniform(0.5, 1.41)
        s = max(abs(w.real), abs(w.imag))
        k = int(np.floor(np.log2(s))) + 1
        w = w / 2.0 ** k          # exact
        for n in ns:
            hm.hm_cpow(w.real, w.imag, n, ctypes.byref(pr), ctypes.byref(pi), ctypes.byref(E))
            got = mpmath.mpc(pr.value, pi.value) * mpmath.mpf(2) ** E.value
            exact = mpmath.mpc(w.real, w.imag) ** n
            rel = abs(got - exact) / abs(exact)
            assert rel <= 2.0 ** -52, (w, n, float(rel))
            mx = max(abs(pr.value), abs(pi.value))
            assert n == 0 or 0.5 <= mx < 1.0


def _normalised_w(rng):
    t = rng.uniform(0, 2 * np.pi)
    w = complex(np.cos(t), np.sin(t)) * rng.uniform(0.5, 1.41)
    k = int(np.floor(np.log2(max(abs(w.real), abs(w.imag))))) + 1
    return w / 2.0 ** k


def _cdd(rng):
    """A complex double-double with max(|re|, |im|) in [1/2, 1); arguments near
    +-45 degrees are included (heavy cancellation in Re x^2)."""
    import mpmath
    t = rng.uniform(0, 2 * np.pi) if rng.random() < 0.7 else np.pi / 4 * rng.choice([1, 3, 5, 7]) + rng.normal(0, 1e-9)
    rad = rng.uniform(0.5, 1.41)
    x = mpmath.mpc(mpmath.cos(t), mpmath.sin(t)) * rad
    s = max(abs(x.real), abs(x.imag))
    x = x / mpmath.mpf(2) ** (int(mpmath.floor(mpmath.log(s, 2))) + 1)
    rh = float(x.real); rl = float(x.real - rh)
    ih = float(x.imag); il = float(x.imag - ih)
    return np.array([rh, rl, ih, il])


def test_cdd_square_and_product_against_mpmath(hm):
    """Unrounded double-double results: normwise error <= 2^-100 |result|."""
    import mpmath
    mpmath.mp.prec = 300
    rng = np.random.default_rng(6)
    out = np.zeros(4)
    dp = ctypes.POINTER(ctypes.c_double)
    for _ in range(3000):
        x = _cdd(rng)
        xm = mpmath.mpc(mpmath.mpf(x[0]) + mpmath.mpf(x[1]), mpmath.mpf(x[2]) + mpmath.mpf(x[3]))
        hm.hm_cdd_sqr(x.ctypes.data_as(dp), out.ctypes.data_as(dp))
        got = mpmath.mpc(mpmath.mpf(out[0]) + mpmath.mpf(out[1]), mpmath.mpf(out[2]) + mpmath.mpf(out[3]))
        ref = xm * xm
        assert abs(got - ref) <= 2.0 ** -100 * abs(ref), (x, float(abs(got - ref) / abs(ref)))
        w = _normalised_w(rng)
        hm.hm_cdd_mul_d(x.ctypes.data_as(dp), w.real, w.imag, out.ctypes.data_as(dp))
        got = mpmath.mpc(mpmath.mpf(out[0]) + mpmath.mpf(out[1]), mpmath.mpf(out[2]) + mpmath.mpf(out[3]))
        ref = xm * mpmath.mpc(w.real, w.imag)
        assert abs(got - ref) <= 2.0 ** -100 * abs(ref), (x, w, float(abs(got - ref) / abs(ref)))


def test_chunk_start_powers_against_mpmath(hm):
    """w^(c C) from an anchor and chained products: relative error below
    3 kAnchor 2^-53 (kAnchor = 8), whichever c."""
    import mpmath
    mpmath.mp.prec = 256
    rng = np.random.default_rng(7)
    pr, pi, E = ctypes.c_double(), ctypes.c_double(), ctypes.c_longlong()
    C = 512
    worst = 0.0
    for _ in range(150):
        w = _normalised_w(rng)
        for c in [0, 1, 2, 7, 8, 9, 15, 16, 255, 1023, 1953, 2047]:
            hm.hm_chunk_start(w.real, w.imag, c, C, ctypes.byref(pr), ctypes.byref(pi), ctypes.byref(E))
            got = mpmath.mpc(pr.value, pi.value) * mpmath.mpf(2) ** E.value
            exact = mpmath.mpc(w.real, w.imag) ** (c * C)
            rel = float(abs(got - exact) / abs(exact))
            worst = max(worst, rel)
            assert rel <= 3 * 8 * 2.0 ** -53, (w, c, rel)
            mx = max(abs(pr.value), abs(pi.value))
            assert c == 0 or 0.5 <= mx < 1.0        # w^0 is returned as 1


def _mp(v):
    import mpmath
    return mpmath.mpc(mpmath.mpf(v[0]) + mpmath.mpf(v[1]), mpmath.mpf(v[2]) + mpmath.mpf(v[3]))


def test_cdd_unnormalised_low_words(hm):
    """Between renormalisations the powering leaves low words unnormalised, up
    to 2^-46 |x| after four squarings: a square or a product by w then drops at
    most the products of two low words, 2^-92 |x|^2, plus roundings far below
    it; the renormalisation folds the low words in exactly and scales by a
    power of two."""
    import mpmath
    mpmath.mp.prec = 300
    rng = np.random.default_rng(9)
    out = np.zeros(4)
    E = ctypes.c_longlong()
    dp = ctypes.POINTER(ctypes.c_double)
    for _ in range(3000):
        x = _cdd(rng)
        mag = max(abs(x[0]), abs(x[2]))
        x[1] = rng.uniform(-1, 1) * 2.0 ** -46 * mag
        x[3] = rng.uniform(-1, 1) * 2.0 ** -46 * mag
        xm = _mp(x)
        hm.hm_cdd_sqr(x.ctypes.data_as(dp), out.ctypes.data_as(dp))
        ref = xm * xm
        assert abs(_mp(out) - ref) <= 2.0 ** -90 * abs(ref), x
        w = _normalised_w(rng)
        hm.hm_cdd_mul_d(x.ctypes.data_as(dp), w.real, w.imag, out.ctypes.data_as(dp))
        ref = xm * mpmath.mpc(w.real, w.imag)
        assert abs(_mp(out) - ref) <= 2.0 ** -90 * abs(ref), (x, w)
        # renormalisation of a scaled copy: exact, high words normalised, low words below ulp/2
        y = x * 2.0 ** int(rng.integers(-30, 9))
        hm.hm_cdd_renorm(y.ctypes.data_as(dp), out.ctypes.data_as(dp), ctypes.byref(E))
        assert _mp(out) * mpmath.mpf(2) ** E.value == _mp(y)
        assert 0.5 <= max(abs(out[0]), abs(out[2])) < 1.0
        assert abs(out[1]) <= 2.0 ** -53 * abs(out[0]) and abs(out[3]) <= 2.0 ** -53 * abs(out[2])
