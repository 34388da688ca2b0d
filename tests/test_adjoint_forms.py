"""Host checks of the closed forms the adjoint's far levels are built from
(paper_2609_17273_amd/csrc/k_adjoint.hip), written here in numpy FP64 as the
kernel writes them, against the same Gauss-Hermite rule differentiated term by
term.

For a line with y and points x_k carrying cotangents g_k, the kernel's window
sums are A = sum g Re w, B = sum g (Re w + x dRe w/dx + y dRe w/dy) and
C = -sum g dRe w/dy, with the rule's Re w = (y/pi) sum_j W_j / ((x - t_j)^2 + y^2).
Three forms are checked: the per-point one (e, t, 1/d and e^2 of each node
pair), the block-summed one (four sums S0..S3 per pair in s = u + h, combined
once per block) and the u-form of waves with larger y (four sums in u),
for one pair, the three-point rule (a pair and the node at 0, which the block
form reduces to sum g/v and sum g/v^2) and two pairs."""
import numpy as np
import pytest

from test_device_constants import D

RULES = {
    # rule: [(tau, W)] of the pairs, plus the weight of the node at 0
    "one pair": ([(D["XS_GH2_TAU"][0], D["XS_GH2_W"][0])], 0.0),
    "three-point": ([(D["XS_GH3_TAU"][0], D["XS_GH3_W"][0])], D["XS_GH3_W0"]),
    "two pairs": (list(zip(D["XS_GH4_TAU"], D["XS_GH4_W"])), 0.0),
}


def direct(rule, x, y, g):
    """A, B, C from the rule's nodes, each term differentiated directly, and
    the scale of each: the same sums with every term (per point, Re w,
    x dRe w/dx and y dRe w/dy apart) in absolute value.  In the far wing B's
    three terms nearly cancel at every point."""
    pairs, w0 = RULES[rule]
    nodes = [(s * np.sqrt(t), W) for t, W in pairs for s in (1.0, -1.0)]
    if w0:
        nodes.append((0.0, w0))
    re = dx = dy = 0.0
    for t, W in nodes:
        f = 1.0 / ((x - t) ** 2 + y * y)
        re = re + W * y / np.pi * f
        dx = dx + W * y / np.pi * (-2.0 * (x - t)) * f * f
        dy = dy + W / np.pi * f + W * y / np.pi * (-2.0 * y) * f * f
    A = np.sum(g * re)
    B = np.sum(g * (re + x * dx + y * dy))
    C = -np.sum(g * dy)
    a = np.abs(g)
    scale = (np.sum(a * re), np.sum(a * (re + np.abs(x * dx) + np.abs(y * dy))), np.sum(a * np.abs(dy)))
    return np.array([A, B, C]), np.array(scale)


def kernel_pairs(rule, y):
    """The level's pairs as the kernel sets them (tau, K = 2 W / pi); the node
    at 0 is the pair with tau = 0 and weight W_0 / 2."""
    pairs, w0 = RULES[rule]
    out = [(t, 2.0 * W / np.pi) for t, W in pairs]
    if w0:
        out.append((0.0, 2.0 * (0.5 * w0) / np.pi))
    return out


def per_point(rule, x, y, g):
    """The per-point form: per pair e = (u + p)/d, rd = 1/d and
    t = (u/d)(4 tau (p - u)/d - 1), d = u (u + q) + p^2, p = y^2 + tau,
    q = 2 y^2 - 2 tau; sums of g e, g t, g/d and g e^2 weighted by K."""
    u = x * x
    y2 = y * y
    ge = gt = gd = ge2 = 0.0
    for tau, K in kernel_pairs(rule, y):
        p, q = y2 + tau, 2.0 * y2 - 2.0 * tau
        d = u * (u + q) + p * p
        rd = 1.0 / d
        e = (u + p) * rd
        t = (u * rd) * (rd * (u * (-4.0 * tau) + 4.0 * tau * p) - 1.0)
        ge += K * np.sum(g * e)
        gt += K * np.sum(g * t)
        gd += K * np.sum(g * rd)
        ge2 += K * np.sum(g * e * e)
    return finish(y, ge, gt, gd, ge2)


def block(rule, x, y, g):
    """The block-summed form: per pair, in s = u + h (h = y^2 - tau), with
    d = s^2 + c (c = 4 y^2 tau), the sums S0 = sum g/d, S1 = sum g s/d,
    S2 = sum g/d^2, S3 = sum g s/d^2, combined as the kernel combines them;
    the node at 0 (tau = 0) accumulates only S0 = sum g/v^2 and S1 = sum g/v,
    v = u + y^2."""
    u = x * x
    y2 = y * y
    ge = gt = gd = ge2 = 0.0
    for tau, K in kernel_pairs(rule, y):
        h, c, t4 = y2 - tau, 4.0 * y2 * tau, 4.0 * tau
        m = 0.5 * t4
        if tau == 0.0:
            v = u + y2
            gv = g / v
            S0, S1, S2, S3 = np.sum(gv / v), np.sum(gv), 0.0, 0.0
        else:
            s = u + h
            rd = 1.0 / (s * s + c)
            grd = g * rd
            S0, S1, S2, S3 = np.sum(grd), np.sum(grd * s), np.sum(grd * rd), np.sum(grd * rd * s)
        sq = S0 - c * S2
        ge += K * (S1 + m * S0)
        gd += K * S0
        ge2 += K * (sq + 2.0 * m * S3 + m * m * S2)
        gt += K * (t4 * ((2.0 * y2 + h) * S3 - sq - 2.0 * y2 * h * S2) - (S1 - h * S0))
    return finish(y, ge, gt, gd, ge2)


def u_form(rule, x, y, g):
    """The one-pair form of waves with larger y: four sums in u = x^2 taken
    directly, S0 = sum g/d, U1 = sum g u/d, U2 = sum g u/d^2 and
    U3 = sum g u^2/d^2, with e^2 = 1/d + 4 tau u/d^2 (from
    d = u^2 + q u + p^2 and 2 p - q = 4 tau):
    sum g e = U1 + p S0, sum g e^2 = S0 + 4 tau U2,
    sum g t = 4 tau (p U2 - U3) - U1."""
    u = x * x
    y2 = y * y
    ge = gt = gd = ge2 = 0.0
    for tau, K in kernel_pairs(rule, y):
        p, q = y2 + tau, 2.0 * y2 - 2.0 * tau
        rd = 1.0 / (u * (u + q) + p * p)
        gr = g * rd
        v = gr * rd * u
        S0, U1, U2, U3 = np.sum(gr), np.sum(gr * u), np.sum(v), np.sum(v * u)
        ge += K * (U1 + p * S0)
        gd += K * S0
        ge2 += K * (S0 + 4.0 * tau * U2)
        gt += K * (4.0 * tau * (p * U2 - U3) - U1)
    return finish(y, ge, gt, gd, ge2)


def finish(y, ge, gt, gd, ge2):
    y2 = y * y
    w = ge + 2.0 * y2 * gd - 4.0 * y2 * ge2  # dRe w/dy summed against g
    return y * ge, y * (ge + 2.0 * gt) + y * w, -w


LEVEL_RHO = {"one pair": 9.0e6, "three-point": 4.5e4, "two pairs": 4000.0}


@pytest.mark.parametrize("rule", list(RULES))
@pytest.mark.parametrize("y", [1e-6, 1e-3, 0.3, 5.0, 40.0, 300.0, 3e4])
def test_far_level_forms_match_the_rule(rule, y):
    """Both forms equal the rule's direct derivatives over a window of points
    in the level's region (|z|^2 >= its bound; the block form as the kernel
    uses it, for y^2 at most half the bound), with cotangents of both signs
    and with positive ones."""
    rng = np.random.default_rng(11)
    R = LEVEL_RHO[rule]
    X = np.sqrt(max(R * 1.001 - y * y, 0.0))
    x = np.concatenate([np.linspace(X, 40 * X, 300), -np.linspace(X, 40 * X, 300)])
    for g in (rng.standard_normal(x.size), np.abs(rng.standard_normal(x.size))):
        ref, scale = direct(rule, x, y, g)
        pp = np.array(per_point(rule, x, y, g))
        assert np.all(np.abs(pp - ref) <= 1e-12 * scale), (rule, y, pp, ref)
        uf = np.array(u_form(rule, x, y, g))
        assert np.all(np.abs(uf - ref) <= 1e-12 * scale), (rule, y, uf, ref)
        if y * y <= 0.5 * R:
            bk = np.array(block(rule, x, y, g))
            assert np.all(np.abs(bk - ref) <= 1e-11 * scale), (rule, y, bk, ref)


def test_node_at_zero_is_a_pair_with_tau_zero():
    """The per-point pair formula with tau = 0 and weight W_0 / 2 gives the
    node at 0's Re w, x dRe w/dx and dRe w/dy: e = 1/v, 1/d = 1/v^2,
    t = -u/v^2 (v = u + y^2)."""
    x = np.linspace(-300.0, 300.0, 601)
    y = 0.7
    u, v = x * x, x * x + y * y
    p, q = y * y, 2.0 * y * y
    d = u * (u + q) + p * p
    assert np.allclose(d, v * v, rtol=1e-15, atol=0)
    assert np.allclose((u + p) / d, 1.0 / v, rtol=1e-15, atol=0)
    t = (u / d) * ((1.0 / d) * 0.0 - 1.0)
    assert np.allclose(t, -u / (v * v), rtol=1e-15, atol=0)
