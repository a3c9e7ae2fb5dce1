"""The library's host FP64 cosmology (csrc/cosmo.cpp, built here with g++) against the oracle's
scipy quadrature: two independent implementations of the same integrals."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

from oracle.cosmology import Cosmology, schedule

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    out = os.path.join(tempfile.mkdtemp(), "libcosmo_test.so")
    src = [os.path.join(ROOT, "tests", "cosmo_driver.cpp"), os.path.join(ROOT, "paper_1712_06121_amd", "csrc", "cosmo.cpp")]
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", out, *src], check=True)
    return ctypes.CDLL(out)


@pytest.mark.parametrize("om,ol,s8", [(1.0, 0.0, 0.8), (0.3, 0.7, 0.8), (0.25, 0.75, 0.9)])
def test_schedule_factors_match_oracle(lib, om, ol, s8):
    a, ah = schedule(0.02, 1.0, 50)
    a0 = np.ascontiguousarray(a[:-1])
    a1 = np.ascontiguousarray(a[1:])
    n = len(a0)
    kick, drift, D, f = (np.empty(n) for _ in range(4))
    amp = ctypes.c_double()
    p = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    lib.cosmo_eval.argtypes = [ctypes.c_double] * 5 + [ctypes.c_int] + [ctypes.c_void_p] * 6 + [ctypes.c_void_p]
    lib.cosmo_eval(om, ol, 0.7, s8, 1.0, n, p(a0), p(a1), p(kick), p(drift), p(D), p(f), ctypes.byref(amp))
    c = Cosmology(om, ol, h=0.7, sigma8=s8)
    for i in range(0, n, 7):
        assert kick[i] == pytest.approx(c.kick_factor(a0[i], a1[i]), rel=1e-11)
        assert drift[i] == pytest.approx(c.drift_factor(a0[i], a1[i]), rel=1e-11)
        assert D[i] == pytest.approx(c.D(a1[i]), rel=1e-11)
        assert f[i] == pytest.approx(c.f(a1[i]), rel=1e-10)
    assert amp.value == pytest.approx(c.amplitude, rel=1e-8)
