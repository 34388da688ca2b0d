"""Host checks of the constants the device Faddeeva function is built from
(paper_2609_17273_amd/csrc/faddeeva_table.h), against library routines: the
Gauss-Hermite nodes and weights against numpy's rule, and the error bounds
the kernels' region thresholds rely on against scipy.special.wofz and
mpmath.  The formulas are evaluated here in numpy FP64 exactly as the kernels
write them."""
import os
import re

import mpmath as mp
import numpy as np
import pytest
from scipy.special import wofz

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2609_17273_amd", "csrc", "faddeeva_table.h")


def _defs():
    text = open(HDR).read()
    out = {}
    for name, body in re.findall(r"#define (XS_\w+) (.+)", text):
        body = body.strip()
        if body.startswith("{"):
            out[name] = np.array([float.fromhex(v.strip()) for v in body.strip("{} ").split(",")])
        else:
            out[name] = float.fromhex(body)
    return out


D = _defs()


def gh_re(n, x, y):
    """Re w by the n-point Gauss-Hermite rule in node-pair form (odd n: plus
    the node at 0, (y/pi) W_0 / |z|^2)."""
    tau, W = D[f"XS_GH{n}_TAU"], D[f"XS_GH{n}_W"]
    u = x * x
    s = 0.0
    for t, w in zip(tau, W):
        p = y * y + t
        s = s + w * (u + p) / ((u - p) ** 2 + 4 * y * y * u)
    if n % 2:
        s = s + 0.5 * D[f"XS_GH{n}_W0"] / (u + y * y)
    return 2 * y / np.pi * s


def poly3_re(x, y):
    """The three-point rule as the gather's FP64 fraction N(s)/D(s) in
    s = |z|^2 - tau, coefficients formed as make_poly3 forms them (c0 = 1)."""
    tau, W, W0 = D["XS_GH3_TAU"][0], D["XS_GH3_W"][0], D["XS_GH3_W0"]
    y2 = y * y
    k = y * (2.0 / np.pi)
    cw, e, c = k * W, 0.5 * k * W0, 4.0 * y2 * tau
    n2, n1, n0 = cw + e, 3.0 * cw * tau, 2.0 * cw * tau * tau + e * c
    s = x * x + (y2 - tau)
    return (n2 * s + n1) * s + n0, ((s + tau) * s + c) * s + c * tau


def weideman(n, z):
    L, a = D[f"XS_WM{n}_L"], D[f"XS_WM{n}_A"]
    q = 1.0 / (L - 1j * z)
    Z = (L + 1j * z) * q
    p = np.zeros_like(z)
    for c in a[::-1]:
        p = p * Z + c
    return 2 * p * q * q + q / np.sqrt(np.pi)


@pytest.mark.parametrize("n", [2, 3, 4, 6, 8, 12])
def test_gauss_hermite_nodes_match_numpy(n):
    t, w = np.polynomial.hermite.hermgauss(n)
    pos = t > 0
    assert np.allclose(np.sort(t[pos] ** 2), D[f"XS_GH{n}_TAU"], rtol=1e-14, atol=0)
    assert np.allclose(w[pos][np.argsort(t[pos])], D[f"XS_GH{n}_W"], rtol=1e-12, atol=0)
    # the weights add up to sqrt(pi), the pairs' half each
    w0 = D[f"XS_GH{n}_W0"] if n % 2 else 0.0
    if n % 2:
        assert abs(w0 - w[np.abs(t) < 1e-12][0]) < 1e-14
    assert abs(2 * D[f"XS_GH{n}_W"].sum() + w0 - np.sqrt(np.pi)) < 1e-14


def test_three_point_rule_exact_on_low_moments():
    """The three-point rule integrates t^k e^{-t^2} exactly for k <= 5
    (moments sqrt(pi), sqrt(pi)/2, 3 sqrt(pi)/4 for k = 0, 2, 4) and misses
    k = 6 (15 sqrt(pi)/8) by 3 sqrt(pi)/4, the coefficient of its leading
    error term 1/z^7."""
    t = np.sqrt(D["XS_GH3_TAU"][0])
    W, W0 = D["XS_GH3_W"][0], D["XS_GH3_W0"]
    q = lambda k: W0 * (0.0 ** k) + 2 * W * t ** k
    sp = np.sqrt(np.pi)
    for k, m in ((0, sp), (2, sp / 2), (4, 3 * sp / 4)):
        assert abs(q(k) - m) < 1e-14 * m, k
    assert abs((15 * sp / 8 - q(6)) - 3 * sp / 4) < 1e-13


def _grid(xmax, ymax, nx=1201, ny=301):
    xs = np.linspace(-xmax, xmax, nx)
    ys = np.concatenate([[0.0, 1e-6, 1e-3], np.linspace(0.01, ymax, ny)])
    X, Y = np.meshgrid(xs, ys)
    return X + 1j * Y


@pytest.mark.parametrize("n,bound", [(24, 5e-10), (40, 3e-14)])
def test_weideman_relative_error(n, bound):
    Z = _grid(25.0, 12.0)
    err = np.abs(weideman(n, Z) - wofz(Z)) / np.abs(wofz(Z))
    assert err.max() < bound, err.max()


def test_weideman_against_mpmath():
    rng = np.random.default_rng(7)
    for _ in range(40):
        z = complex(rng.uniform(-9, 9), rng.uniform(0, 9))
        ref = complex(mp.exp(-mp.mpc(z) ** 2) * mp.erfc(-1j * mp.mpc(z)))
        assert abs(complex(weideman(40, np.array([z]))[0]) - ref) <= 3e-14 * abs(ref)
        assert abs(complex(weideman(24, np.array([z]))[0]) - ref) <= 5e-10 * abs(ref)


# (rule, rho threshold, bound on the relative error of Re w where Re w > 1e-9)
FP32_BANDS = [(2, 900.0, 4e-6), (4, 64.0, 1.1e-6), (6, 36.0, 2e-7)]
FP64_BANDS = [(2, 9.0e6, 1e-13), (3, 4.5e4, 1e-13), (4, 4000.0, 1e-13), (6, 400.0, 1e-13),
              (8, 144.0, 1e-13), (12, 64.0, 1e-13)]


@pytest.mark.parametrize("n,rho,bound", FP32_BANDS + FP64_BANDS)
def test_gauss_hermite_band_error(n, rho, bound):
    r = np.sqrt(rho)
    # points on and just outside the band edge, plus a far sample
    th = np.linspace(0.0, np.pi / 2, 721)
    pts = []
    for scale in (1.0, 1.01, 1.1, 2.0, 10.0):
        pts.append(scale * r * (np.cos(th) + 1j * np.sin(th)))
    Z = np.concatenate(pts)
    Z = Z[Z.imag >= 0]
    ex = wofz(Z).real
    keep = ex > 1e-9
    got = gh_re(n, Z.real, Z.imag)
    err = np.abs(got[keep] - ex[keep]) / ex[keep]
    assert err.max() < bound, (n, rho, err.max())


def test_three_point_fraction_matches_rule_and_wofz():
    """The gather's three-point fraction (rows wholly at |z|^2 >= 4.5e4)
    against the rule summed term by term and against Re w, on and beyond
    the band edge for every direction of z, including y near 0 and y large."""
    th = np.linspace(0.0, np.pi / 2, 721)
    Z = np.concatenate([sc * np.sqrt(4.5e4) * (np.cos(th) + 1j * np.sin(th))
                        for sc in (1.0, 1.01, 1.1, 2.0, 10.0, 100.0, 1e3)])
    Z = np.concatenate([Z, np.array([complex(x, y) for x in (212.2, 1e3, 1e5, 1e8)
                                     for y in (1e-12, 1e-6, 1e-3, 1.0, 1e3, 1e6)])])
    N, Dn = poly3_re(Z.real, Z.imag)
    frac = N / Dn
    ref = gh_re(3, Z.real, Z.imag)
    keep = ref > 0
    assert np.max(np.abs(frac[keep] - ref[keep]) / ref[keep]) < 2e-15
    ex = wofz(Z).real
    keep = ex > 1e-300
    assert np.max(np.abs(frac[keep] - ex[keep]) / ex[keep]) < 1e-13


def poly2_re(x, y):
    """The four-point rule as the gather's FP64 fraction N(s)/D(s) in
    s = |z|^2 - tau_1, coefficients formed as make_poly2 forms them (c0 = 1)."""
    t1, t2 = D["XS_GH4_TAU"]
    w1, w2 = D["XS_GH4_W"]
    y2 = y * y
    k = y * (2.0 / np.pi)
    cw1, cw2 = k * w1, k * w2
    d, c1 = t1 - t2, 4.0 * y2 * t1
    q = d * d + 4.0 * y2 * t2
    e1, e2 = 2.0 * t1, t1 + t2
    n3, n2 = cw1 + cw2, cw1 * (2.0 * d + e1) + cw2 * e2
    n1, n0 = cw1 * (q + 2.0 * d * e1) + cw2 * c1, cw1 * e1 * q + cw2 * e2 * c1
    d3, d2, d1, d0 = 2.0 * d, q + c1, 2.0 * d * c1, c1 * q
    s = x * x + (y2 - t1)
    N = ((n3 * s + n2) * s + n1) * s + n0
    Dn = (((s + d3) * s + d2) * s + d1) * s + d0
    return N, Dn


def test_two_pair_fraction_matches_rule_and_wofz():
    """The gather's two-pair fraction (rows wholly at |z|^2 >= 4000) against
    the four-point rule summed term by term and against Re w, on and beyond
    the band edge for every direction of z, including y near 0 and y large."""
    th = np.linspace(0.0, np.pi / 2, 721)
    Z = np.concatenate([sc * np.sqrt(4000.0) * (np.cos(th) + 1j * np.sin(th))
                        for sc in (1.0, 1.01, 1.1, 2.0, 10.0, 100.0, 1e3)])
    Z = np.concatenate([Z, np.array([complex(x, y) for x in (63.3, 1e3, 1e5, 1e8)
                                     for y in (1e-12, 1e-6, 1e-3, 1.0, 1e3, 1e6)])])
    N, Dn = poly2_re(Z.real, Z.imag)
    frac = N / Dn
    ref = gh_re(4, Z.real, Z.imag)
    keep = ref > 0
    assert np.max(np.abs(frac[keep] - ref[keep]) / ref[keep]) < 2e-15
    ex = wofz(Z).real
    keep = ex > 1e-300
    assert np.max(np.abs(frac[keep] - ex[keep]) / ex[keep]) < 1e-13
