"""The library's host-only FP64 arithmetic under AddressSanitizer and UndefinedBehavior-
Sanitizer on the CPU: csrc/host_math.cpp (k-bin geometry, the time grid of eq. (P-final))
and csrc/background.cpp (H(a), s, the relativistic neutrino background of eq.
(relativistic)), built with g++ and the sanitizers into a small driver
(tests/host_check/host_math_check.cpp) and compared with the oracle:

* bin edges, mode counts and the table of bins per integer |n|^2 bit-exact, mean |k| to
  rounding, against oracle.pm (brute-force pinned there);
* H(a) against oracle.background for matter + Lambda and the relativistic background;
* the sub-nodes, s(a_now) - s(a_q) and weights of the time grid against
  oracle.response.sub_grid, whose weight is the trapezoid weight in ln a (the library's
  carries the factor (3/2) Omega_M H0^2 / (a H) of eq. (P-final) as well).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import background as obg
from oracle import pm as opm
from oracle import response as oresp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1209_0461_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("hostcheck") / "host_math_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g"] + SAN + [
        os.path.join(ROOT, "tests", "host_check", "host_math_check.cpp"),
        os.path.join(CSRC, "host_math.cpp"), os.path.join(CSRC, "background.cpp"),
        "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def _f(x):
    return format(float(x), ".17g")


def _run(driver, requests):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver], input="\n".join(requests) + "\n", capture_output=True,
                       text=True, env=env, timeout=300)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "ERROR:" not in r.stderr, \
        r.stderr[-3000:]
    out = []
    for line in r.stdout.splitlines():
        name, *vals = line.split()
        out.append((name, np.array([float(v) for v in vals])))
    return out


@pytest.mark.parametrize("n,box,nb", [(8, 32.0, 5), (32, 128.0, 32), (64, 256.0, 48),
                                      (128, 256.0, 40), (256, 512.0, 64)])
def test_bin_geometry_matches_oracle(driver, n, box, nb):
    res = dict(_run(driver, [f"bins {n} {_f(box)} {nb}"]))
    edges, counts, kmean = opm.bin_geometry(n, box, nb)
    assert np.array_equal(res["edges"], edges)
    assert np.array_equal(res["counts"], counts)
    ok = counts > 0
    assert np.allclose(res["kmean"][ok], kmean[ok], rtol=1e-12, atol=0)
    assert np.all(res["kmean"][~ok] == 0)
    n2 = np.arange(3 * n * n // 4 + 1)
    table = opm.bin_of_n2(n2, edges)
    assert np.array_equal(res["table"][1:], table[1:])
    assert np.array_equal(res["nonempty"], np.flatnonzero(ok))


def _bg_args(rel, om, h, masses):
    """(request text, oracle background) for three equal masses or a list of species."""
    massive = [m for m in masses if m > 0]
    distinct = sorted(set(massive))
    n_massless = len(masses) - len(massive)
    if len(distinct) == 1 and len(massive) > 1:
        spec = f"{len(massive)} {n_massless} 1 {_f(distinct[0])}"
    else:
        spec = f"1 {n_massless} {len(massive)} " + " ".join(_f(m) for m in massive)
    return f"{int(rel)} {_f(om)} {_f(h)} {spec}", (obg.Background(om, h, masses) if rel else None)


@pytest.mark.parametrize("rel,masses", [(False, (0.1, 0.1, 0.1)), (True, (0.1, 0.1, 0.1)),
                                        (True, (0.0, 0.049, 0.051)),
                                        (True, (0.022, 0.024, 0.054))])
def test_hubble_rate_matches_oracle(driver, rel, masses):
    om, h = 0.3, 0.7
    a = np.geomspace(1e-4, 1.0, 40)
    spec, bg = _bg_args(rel, om, h, masses)
    res = dict(_run(driver, [f"hubble {spec} {len(a)} " + " ".join(_f(x) for x in a)]))
    ref = np.array([obg.hubble_rate(x, om, bg) for x in a])
    assert np.allclose(res["hubble"], ref, rtol=1e-10, atol=0)


@pytest.mark.parametrize("rel,masses,Q,J", [(False, (0.1, 0.1, 0.1), 8, 12),
                                            (False, (0.2, 0.2, 0.2), 1, 6),
                                            (True, (0.022, 0.024, 0.054), 4, 9)])
def test_time_grid_matches_oracle(driver, rel, masses, Q, J):
    om, h = 0.3, 0.7
    nodes = np.geomspace(0.01, 0.6, J)
    spec, bg = _bg_args(rel, om, h, masses)
    res = dict(_run(driver, [f"grid {spec} {Q} {J} " + " ".join(_f(x) for x in nodes)]))
    g = oresp.sub_grid(nodes, Q, om, bg)
    assert np.allclose(res["a"], g["a"], rtol=1e-14, atol=0)
    assert np.allclose(res["ds"], g["ds"], rtol=1e-9, atol=1e-12 * g["ds"][0])
    pref = 1.5 * om * obg.H0 ** 2
    measure = pref / (g["a"] * obg.hubble_rate(g["a"], om, bg))
    assert np.allclose(res["w"], g["w"] * measure, rtol=1e-10, atol=0)
