"""Pins of the oracle's reverse pass (differentiable form) against central
finite differences of the oracle's forward functions, which are themselves
pinned in test_oracle_pins.py.  Every check is a directional derivative:
<cotangent, J tangent> by FP64 central differences against
<J^T cotangent, tangent> from the hand-written reverse pass.  Inputs avoid
kinks (contact onset, stick/slip switch, alpha clamp) except where a test
is about a branch, and then the perturbation stays inside the branch.
"""
import numpy as np
import pytest

from paper_2504_00745_amd import workloads as wl
from test_oracle_pins import random_bed, small_cfg


def _fd(f, h):
    return (f(h) - f(-h)) / (2 * h)


def _bed(seed, n=1800, slide_mu=0.5):
    cfg = small_cfg(nc=[10, 10, 10], cell=0.032, walls=0x3F, mu=slide_mu)
    x, r = random_bed(n, [0.32, 0.32, 0.32], 0.005, 0.015, seed, overlap=1.15)
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    v = rng.normal(0, 0.2, x.shape)
    return cfg, x, v, r, rng


@pytest.mark.parametrize("mu", [0.5, 5.0, 0.01])
def test_contact_vjp_directional(orc, mu):
    """mu = 5 keeps most contacts sticking, 0.01 makes most slide."""
    cfg, x, v, r, rng = _bed(1, slide_mu=mu)
    # a few granules pressed into walls too
    x[0, :5] = r[:5] * 0.9
    x[2, 5:10] = 0.32 - r[5:10] * 0.95
    gF = rng.normal(0, 1, x.shape)
    dx = rng.normal(0, 1, x.shape)
    dv = rng.normal(0, 1, v.shape)
    gx, gv, gmu = orc.contact_vjp(cfg, x, v, r, gF)
    _, _, nc, ns = orc.contact_forces(cfg, x, v, r)
    assert nc.sum() > 300
    if mu == 0.01:
        assert ns.sum() > 0.5 * nc.sum()

    def loss_x(h):
        return np.sum(gF * orc.contact_forces(cfg, x + h * dx, v, r)[0])

    def loss_v(h):
        return np.sum(gF * orc.contact_forces(cfg, x, v + h * dv, r)[0])

    def loss_mu(h):
        return np.sum(gF * orc.contact_forces(dict(cfg, mu=mu + h), x, v, r)[0])

    hx = 1e-9  # far below every overlap, so no contact starts or ends
    assert _fd(loss_x, hx) == pytest.approx(np.sum(gx * dx), rel=1e-5)
    assert _fd(loss_v, 1e-6) == pytest.approx(np.sum(gv * dv), rel=1e-6)
    assert _fd(loss_mu, mu * 1e-6) == pytest.approx(gmu, rel=1e-6, abs=1e-12)


def test_drag_vjp_directional(orc):
    cfg = small_cfg(c_drag=30.0)
    rng = np.random.Generator(np.random.PCG64(3))
    n = 500
    r = rng.uniform(0.003, 0.01, n)
    v = rng.normal(0, 0.1, (3, n))
    uat = rng.normal(0, 0.1, (3, n))
    af = rng.uniform(0.3, 1.0, n)
    gF = rng.normal(0, 1, (3, n))
    gv, guat, gaf, gcd = orc.drag_vjp(cfg, r, v, uat, af, gF)
    dv, du, da = rng.normal(0, 1, (3, n)), rng.normal(0, 1, (3, n)), rng.normal(0, 1, n)

    def L(h, which):
        vv, uu, aa, cc = v, uat, af, 30.0
        if which == "v": vv = v + h * dv
        if which == "u": uu = uat + h * du
        if which == "a": aa = af + h * da
        if which == "c": cc = 30.0 + h
        return np.sum(gF * orc.drag(dict(cfg, c_drag=cc), r, vv, uu, aa))

    assert _fd(lambda h: L(h, "v"), 1e-6) == pytest.approx(np.sum(gv * dv), rel=1e-8)
    assert _fd(lambda h: L(h, "u"), 1e-6) == pytest.approx(np.sum(guat * du), rel=1e-8)
    assert _fd(lambda h: L(h, "a"), 1e-6) == pytest.approx(np.sum(gaf * da), rel=1e-8)
    assert _fd(lambda h: L(h, "c"), 1e-4) == pytest.approx(gcd, rel=1e-8)


def test_g2p_and_p2g_vjp_directional(orc):
    cfg = small_cfg()
    G = 16 ** 3
    rng = np.random.Generator(np.random.PCG64(4))
    n = 400
    x = rng.uniform(0.0, 0.32, (3, n))
    r = rng.uniform(0.003, 0.009, n)
    v = rng.normal(0, 0.2, (3, n))
    u = rng.normal(0, 0.1, (3, G))
    A = rng.uniform(0.0, 0.6, G)
    A[::7] = 0.9  # some nodes above the 0.74 clamp
    guat = rng.normal(0, 1, (3, n))
    gaf = rng.normal(0, 1, n)
    gx, gA = orc.g2p_vjp(cfg, x, u, A, guat, gaf)
    dx = rng.normal(0, 1, (3, n))
    dA = rng.normal(0, 1, G)

    def L(h, which):
        xx = x + h * dx if which == "x" else x
        AA = A + h * dA if which == "A" else A
        ua, af = orc.g2p(cfg, xx, u, alpha_real=AA)
        return np.sum(guat * ua) + np.sum(gaf * af)

    assert _fd(lambda h: L(h, "x"), 1e-9) == pytest.approx(np.sum(gx * dx), rel=1e-6)
    assert _fd(lambda h: L(h, "A"), 1e-7) == pytest.approx(np.sum(gA * dA), rel=1e-8)
    assert np.all(gA[::7] == 0.0)  # clamped nodes pass no gradient
    # P2G
    ga = rng.normal(0, 1, G)
    gm = rng.normal(0, 1, (3, G))
    gx2, gv2 = orc.p2g_vjp(cfg, x, v, r, ga, gm)
    dv = rng.normal(0, 1, (3, n))

    def Lp(h, which):
        xx = x + h * dx if which == "x" else x
        vv = v + h * dv if which == "v" else v
        a, m = orc.p2g_real(cfg, xx, vv, r)
        return np.sum(ga * a) + np.sum(gm * m)

    assert _fd(lambda h: Lp(h, "x"), 1e-9) == pytest.approx(np.sum(gx2 * dx), rel=1e-6)
    assert _fd(lambda h: Lp(h, "v"), 1e-6) == pytest.approx(np.sum(gv2 * dv), rel=1e-8)


def _c4_small(n=3000, steps=12):
    d = wl.make("c4", n_override=n)
    return d["params"], d["x"], d["v"], d["r"], d["u"], steps


def test_rollout_gradients_match_central_differences(orc):
    """dL/dmu, dL/dC_d and directional derivatives in v0 of the rollout
    loss L = sum |P|^2 against central differences with h = 1e-6 max(|theta|,1);
    a sample whose contact / sliding / clamp sets differ between theta +- h
    straddles a kink and is excluded (at most 1 of 4 here)."""
    cfg, x, v, r, u, steps = _c4_small()
    L0, gv, gmu, gcd = orc.rollout_vjp(cfg, x, v, r, u, steps)
    Lr, _ = orc.rollout(cfg, x, v, r, u, steps)
    assert L0 == pytest.approx(Lr, rel=1e-14)
    rng = np.random.Generator(np.random.PCG64(9))
    checks = 0
    for which in ("mu", "cd", "v", "v", "v"):
        if which == "mu":
            h = 1e-6 * max(cfg["mu"], 1)
            f = lambda s: orc.rollout(dict(cfg, mu=cfg["mu"] + s * h), x, v, r, u, steps)
            want = gmu
        elif which == "cd":
            h = 1e-6 * max(cfg["c_drag"], 1)
            f = lambda s: orc.rollout(dict(cfg, c_drag=cfg["c_drag"] + s * h), x, v, r, u, steps)
            want = gcd
        else:
            dv = rng.normal(0, 1, v.shape)
            dv /= np.linalg.norm(dv)
            h = 1e-6 * max(np.linalg.norm(v), 1)
            f = lambda s: orc.rollout(cfg, x, v + s * h * dv, r, u, steps)
            want = np.sum(gv * dv)
        (Lp, sp), (Lm, sm) = f(1), f(-1)
        if sp != sm:
            continue
        fd = (Lp - Lm) / (2 * h)
        # FD round-off ~ eps L / h; tolerance 1e-4 of the gradient plus that floor
        assert fd == pytest.approx(want, rel=1e-4, abs=20 * np.finfo(float).eps * L0 / h), which
        checks += 1
    assert checks >= 4
    # the parameters matter: sensitivities well above the FD round-off floor
    assert abs(gmu * cfg["mu"]) > 1e-5 * L0
    assert abs(gcd * cfg["c_drag"]) > 1e-5 * L0
