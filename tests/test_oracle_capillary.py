"""Pins of the oracle's capillary (concentration-gradient) pair force, Sec. 5.4:
the liquid-bridge force against its energy and against the textbook contact
limit, the rupture range, the moisture curve's stated properties, Newton's
third law and the cell list against O(N^2) enumeration.

Parity unpinned: the shape of the moisture curve Gamma between its zeros and
its peak (the paper fits a Bezier curve whose control points it does not
print); only Gamma(0) = Gamma(1) = 0 and the peak at the maximum absorption
ratio are pinned.
"""
import itertools
import math

import numpy as np
import pytest

CAP = dict(sigma=0.072, vbridge=1e-4, sr_peak=0.3)


def test_bridge_force_is_the_energy_slope(orc):
    """F^st = dE/ds of the bridge energy (cos theta = 1): the energy rises with
    the separation, so the bridge pulls the pair together with F^st > 0."""
    for rb in (5e-4, 1e-3, 3e-3):
        _, dr = orc.bridge(CAP, rb)
        for s in (0.01 * dr, 0.2 * dr, 0.9 * dr):
            h = 1e-6 * s
            fd = (orc.bridge_energy(CAP, rb, s + h) - orc.bridge_energy(CAP, rb, s - h)) / (2 * h)
            assert fd > 0 and abs(orc.fst(CAP, rb, s) - fd) <= 1e-6 * fd


def test_bridge_force_contact_limit_and_decay(orc):
    """As s -> 0 the bridge pulls with 2 pi sigma r (the classical capillary
    force between touching spheres at zero contact angle); it decays with s."""
    for rb in (5e-4, 1e-3, 3e-3):
        f0 = orc.fst(CAP, rb, 1e-13)
        assert abs(f0 - 2 * math.pi * 0.072 * rb) <= 1e-6 * f0
        _, dr = orc.bridge(CAP, rb)
        vals = [orc.fst(CAP, rb, s) for s in np.linspace(0.05, 1.0, 20) * dr]
        assert all(a > b > 0 for a, b in zip(vals, vals[1:]))


def test_bridge_volume_and_rupture_distance(orc):
    """V* = 0.01 % of the volume of a sphere of the pair's mean radius; d_r =
    V*^(1/3) + 0.1 V*^(2/3)."""
    rb = 1e-3
    V, dr = orc.bridge(CAP, rb)
    assert math.isclose(V, 1e-4 * 4.0 / 3.0 * math.pi * rb ** 3, rel_tol=1e-15)
    assert math.isclose(dr, V ** (1 / 3) + 0.1 * V ** (2 / 3), rel_tol=1e-14)
    assert 7.48e-5 < dr < 7.49e-5


def test_moisture_curve_properties(orc):
    """Gamma is zero when dry (sr = 0) and when saturated (sr = 1), one at the
    maximum absorption ratio, below one elsewhere, continuous at the peak."""
    assert orc.gamma(CAP, 0.0) == 0.0 and orc.gamma(CAP, 1.0) == 0.0
    assert orc.gamma(CAP, -0.1) == 0.0 and orc.gamma(CAP, 1.7) == 0.0
    assert orc.gamma(CAP, 0.3) == 1.0
    g = [orc.gamma(CAP, s) for s in np.linspace(0.001, 0.999, 999)]
    assert max(g) <= 1.0 and min(g) > 0.0
    assert abs(orc.gamma(CAP, 0.3 - 1e-9) - orc.gamma(CAP, 0.3 + 1e-9)) < 1e-8
    # a smooth (Bezier) curve has a level tangent at its interior maximum
    h = 1e-5
    assert abs(orc.gamma(CAP, 0.3) - orc.gamma(CAP, 0.3 - h)) < 1e-8
    assert abs(orc.gamma(CAP, 0.3) - orc.gamma(CAP, 0.3 + h)) < 1e-8


def test_pair_range_direction_and_antisymmetry(orc):
    """Zero for touching granules and beyond the rupture distance; inside the
    range the force on i points to j with magnitude Gamma F^st; F_ij = -F_ji
    bit for bit."""
    r = 1e-3
    _, dr = orc.bridge(CAP, r)
    xi = np.array([0.1, 0.1, 0.1])
    e = np.array([0.6, -0.48, 0.64])
    for s, on in ((-1e-6, False), (0.5 * dr, True), (0.999 * dr, True), (1.01 * dr, False)):
        xj = xi + (2 * r + s) * e
        Fi = orc.capillary_pair(CAP, xi, xj, r, r, 0.2, 0.5)
        Fj = orc.capillary_pair(CAP, xj, xi, r, r, 0.5, 0.2)
        assert np.array_equal(Fi, -Fj)
        if not on:
            assert not Fi.any()
            continue
        mag = orc.gamma(CAP, 0.35) * orc.fst(CAP, r, s)
        assert np.allclose(Fi, mag * e, rtol=1e-9)  # attractive: along +e, towards j


def test_cell_list_equals_brute_force(orc):
    """The capillary force of a random polydisperse wet bed through the cell
    list equals the sum over all pairs enumerated O(N^2)."""
    rng = np.random.Generator(np.random.PCG64(9))
    # a jittered 8^3 lattice of near-equal spheres: surface gaps spread over
    # about [-10, 90] um around the ~75 um rupture distance
    m = 8
    g = np.stack(np.meshgrid(*[np.arange(m)] * 3, indexing="ij")).reshape(3, -1).astype(float)
    n = g.shape[1]
    r = rng.uniform(0.98e-3, 1.0e-3, n)
    sp = 2.03e-3
    x = (g + 0.5) * sp + rng.uniform(-1e-5, 1e-5, g.shape)
    box = m * sp
    sr = rng.uniform(0.0, 0.9, n)
    _, drmax = orc.bridge(CAP, 1e-3)
    cell = 2e-3 + drmax + 1e-5
    nc = int(box / cell)
    cfg = dict(n=[8, 8, 8], dx=box / 8, nc=[nc] * 3, cell=cell, kn=1e5, restitution=0.5, kt_ratio=1.0, mu=0.5,
               rho_s=2500.0, eta_f=1e-3, c_drag=0.0, alpha_max=0.74, g=[0, 0, 0], dt=1e-5, walls=0, **CAP)
    F = orc.capillary_forces(cfg, x, r, sr)
    B = np.zeros((3, n))
    bridged = 0
    for i, j in itertools.combinations(range(n), 2):
        d = np.linalg.norm(x[:, i] - x[:, j])
        if d - r[i] - r[j] < 2 * drmax:
            f = orc.capillary_pair(CAP, x[:, i], x[:, j], r[i], r[j], sr[i], sr[j])
            B[:, i] += f
            B[:, j] -= f
            bridged += bool(f.any())
    assert bridged > 50
    assert np.allclose(F, B, rtol=1e-12, atol=1e-20)
    assert np.abs(F.sum(axis=1)).max() <= 1e-12 * np.abs(F).sum()
    # the one-by-one form for sampled granules: the same sums, and the sum of
    # the bridge magnitudes bounds the net force
    idx = rng.choice(n, 40, replace=False)
    Fs, fs = orc.capillary_forces_sample(cfg, x, r, sr, idx)
    assert np.array_equal(Fs, F[:, idx])
    assert np.all(np.linalg.norm(Fs, axis=0) <= fs * (1 + 1e-12)) and (fs > 0).sum() > 10


def test_moisture_ratio_is_water_per_sand_volume(orc):
    """sr = held water + alpha_f / (1 - alpha_f): for a mixture of sand
    volume Vs and free water Vw (alpha_f = Vw / (Vs + Vw)) the second term is
    Vw / Vs; pure sand adds nothing and no sand gives +inf (Gamma = 0)."""
    Vs = np.array([3.0, 1.0, 1.0, 5.0, 1.0])
    Vw = np.array([1.0, 1.0, 3.0, 0.0, 0.0])
    held = np.array([0.0, 0.25, 0.1, 0.2, 0.0])
    sr = orc.moisture_ratio(held, Vw / (Vs + Vw))
    assert np.allclose(sr, held + Vw / Vs, rtol=1e-15, atol=0)
    assert orc.moisture_ratio([0.3], [1.0])[0] == math.inf
    assert orc.gamma(CAP, math.inf) == 0.0


def test_moisture_ratio_of_a_lone_granule(orc):
    """A lone granule at a node centre samples alpha_s = frac 0.59375^3 of
    itself (the pinned G2P), so its moisture ratio is held + (1 - alpha_s) /
    alpha_s: the cell's free water over the granule's share of sand."""
    cfg = dict(n=[16, 16, 16], dx=0.02, nc=[16, 16, 16], cell=0.02, kn=1e5, restitution=0.5, kt_ratio=1.0,
               mu=0.5, rho_s=2500.0, eta_f=1e-3, c_drag=1.0, alpha_max=0.74, g=[0, 0, 0], dt=1e-5, walls=0)
    dx = cfg["dx"]
    r0 = 0.006
    x = np.array([[7.5 * dx], [8.5 * dx], [6.5 * dx]])
    alpha, _ = orc.p2g_fixed(cfg, x, np.zeros((3, 1)), np.array([r0]))
    _, af = orc.g2p(cfg, x, np.zeros((3, 16 ** 3)), alpha_fx=alpha)
    a_s = 4 / 3 * np.pi * r0 ** 3 / dx ** 3 * 0.59375 ** 3
    sr = orc.moisture_ratio([0.15], af)[0]
    assert sr == pytest.approx(0.15 + (1 - a_s) / a_s, rel=1e-7)
