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
    L.hm_cpow.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int,
                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(ctypes.c_longlong)]
    return L


def test_cpow_dd_against_mpmath(hm):
    """w^n with w normalised (max component in [1/2, 1)): relative error <= 2^-51 after rounding."""
    import mpmath
    mpmath.mp.prec = 256
    rng = np.random.default_rng(4)
    pr, pi, E = ctypes.c_double(), ctypes.c_double(), ctypes.c_longlong()
    ns = [0, 1, 2, 3, 7, 64, 952, 1000, 4095, 999_999, 1 << 20, (1 << 30) + 12345]
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
            assert rel <= 2.0 ** -51, (w, n, float(rel))
            mx = max(abs(pr.value), abs(pi.value))
            assert n == 0 or 0.5 <= mx < 1.0
