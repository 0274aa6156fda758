"""Pins of the oracle's wet granules (Sec. 5.3, Eq. 19): the mass with the
water a granule holds, m = V (rho_s + held rho_0), in the contact's damping,
the integrator and the momentum deposit; the held water's volume V held in
the solid fraction alpha_s, in the volume forces (pressure gradient, virtual
mass) and the raised clamp 0.740 (1 + r_max) of alpha_s.

Closed forms: a head-on collision of two equal wet spheres lasts
pi / (omega_n sqrt(1 - zeta^2)) with omega_n = sqrt(k_n / m_eff) of the wet
effective mass and still rebounds at e; a lone wet granule's slip in a
uniform flow decays by (1 - dt beta / m_wet) per step; free fall does not
depend on the mass; the momentum grid holds the wet momentum; a lone wet
granule at a node centre samples alpha_s = frac (1 + held) 0.59375^3; a
uniform pressure gradient pushes a wet granule with -V (1 + held) grad p; a
wet sphere released in still fluid accelerates at
g V (rho_s - rho_0) / (m_wet + rho_0 V (1 + held) / 2) (its water is
neutrally buoyant but adds mass and added mass); held = 0 reduces every wet
form to the pinned dry one bit for bit.
"""
import math

import numpy as np
import pytest

RHO_F = 1000.0


def cfg(**over):
    p = dict(n=[16, 16, 16], dx=0.02, nc=[16, 16, 16], cell=0.02, kn=1e5, restitution=0.5, kt_ratio=1.0,
             mu=0.5, rho_s=2500.0, eta_f=1e-3, c_drag=0.0, alpha_max=0.74, g=[0.0, 0.0, 0.0], dt=1e-5,
             walls=0, rho_f=RHO_F, vmass=0, c_quad=0.0, f_unit=1e-3, drag_model=0)
    p.update(over)
    return p


def test_wet_mass_adds_the_held_water(orc):
    """m_wet - m_dry is the held water's mass held V rho_0; held = 0 is the
    dry mass; with rho_s = 2500 and held = 0.2 the ratio is exactly 1.08."""
    c = cfg()
    r = np.array([0.003, 0.005, 0.01, 0.004])
    held = np.array([0.0, 0.2, 0.35, 1.0])
    m = orc.wet_mass(c, r, held)
    V = 4.0 / 3.0 * math.pi * r ** 3
    assert m[0] == pytest.approx(2500.0 * V[0], rel=1e-15)
    assert np.allclose(m - 2500.0 * V, held * V * RHO_F, rtol=1e-12, atol=0)
    assert m[1] / (2500.0 * V[1]) == pytest.approx(1.08, rel=1e-15)


def _head_on(orc, c, held, dt):
    r0 = 0.01
    v0 = 0.1
    gap = 1e-5
    x = np.array([[0.16 - r0 - gap / 2, 0.16 + r0 + gap / 2], [0.16, 0.16], [0.16, 0.16]])
    v = np.array([[v0, -v0], [0.0, 0.0], [0.0, 0.0]])
    r = np.array([r0, r0])
    m = orc.wet_mass(c, r, np.array([held, held]))
    c = dict(c, dt=dt)
    t_in = t_out = None
    t = 0.0
    for _ in range(400000):
        F, _, nc = orc.contact_forces_wet(c, x, v, r, m)
        touching = nc[0] > 0
        x, v = orc.integrate_wet(c, r, m, F, np.zeros((3, 2)), x, v)
        t += dt
        if touching and t_in is None:
            t_in = t - dt
        if t_in is not None and not touching:
            t_out = t - dt
            break
    return -(v[0, 0] - v[0, 1]) / (2 * v0), t_out - t_in, m[0]


def test_wet_head_on_collision_closed_form(orc):
    """Two equal spheres holding water of 0.4 their volume: the rebound
    ratio is still e (the damping ratio depends on e only) and the contact
    lasts pi / (omega_n sqrt(1 - zeta^2)) with the wet effective mass m/2,
    longer than the dry collision by sqrt(m_wet / m_dry)."""
    c = cfg()
    e, tc, m = _head_on(orc, c, 0.4, 5e-7)
    le = math.log(0.5)
    zeta = -le / math.sqrt(math.pi ** 2 + le * le)
    omega = math.sqrt(1e5 / (m / 2))
    t_exact = math.pi / (omega * math.sqrt(1 - zeta ** 2))
    assert e == pytest.approx(0.5, abs=0.01)
    assert tc == pytest.approx(t_exact, rel=0.003)
    _, tc_dry, m_dry = _head_on(orc, c, 0.0, 5e-7)
    assert tc / tc_dry == pytest.approx(math.sqrt(m / m_dry), rel=0.005)


def test_wet_drag_relaxation_and_free_fall(orc):
    """A lone wet granule in a uniform flow: with the explicit drag force
    beta (u - v), beta = C_d 6 pi eta r alpha_f, its slip shrinks by
    (1 - dt beta / m_wet) per step; under gravity alone it falls as a dry
    one does."""
    c = cfg(c_drag=40.0, dt=1e-4)
    r = np.array([0.004])
    held = np.array([0.3])
    m = orc.wet_mass(c, r, held)
    x = np.array([[0.15], [0.17], [0.13]])
    v = np.zeros((3, 1))
    u = np.array([0.2, -0.1, 0.05])
    af = np.array([0.9])
    beta = 40.0 * 6 * math.pi * 1e-3 * 0.004 * 0.9
    for _ in range(50):
        Fd = orc.drag(c, r, v, u[:, None], af)
        x, v = orc.integrate_wet(c, r, m, np.zeros((3, 1)), Fd, x, v)
    slip = (u[:, None] - v)[:, 0]
    assert np.allclose(slip, u * (1 - c["dt"] * beta / m[0]) ** 50, rtol=1e-12)
    g = cfg(g=[0.0, 0.0, -9.81], dt=1e-3)
    xw, vw = x.copy(), np.zeros((3, 1))
    xd, vd = x.copy(), np.zeros((3, 1))
    md = orc.wet_mass(g, r, np.array([0.0]))
    for _ in range(20):
        xw, vw = orc.integrate_wet(g, r, m, np.zeros((3, 1)), np.zeros((3, 1)), xw, vw)
        xd, vd = orc.integrate_wet(g, r, md, np.zeros((3, 1)), np.zeros((3, 1)), xd, vd)
    assert np.array_equal(vw, vd) and np.array_equal(xw, xd)
    assert vw[2, 0] == pytest.approx(-9.81 * 20e-3, rel=1e-12)


def test_wet_momentum_deposit(orc):
    """The momentum grid of wet granules sums, channel by channel, to the
    integer total of the per-granule deposits rint(frac (rho_s + held rho_0) /
    rho_s v 2^32), i.e. within half a unit per granule of the wet momentum in
    rho_s dx^3 units; the fraction grid sums to the granules' volume with
    their water, sum frac (1 + held), within half a unit per granule."""
    c = cfg()
    rng = np.random.Generator(np.random.PCG64(3))
    n = 300
    x = rng.uniform(0.02, 0.30, (3, n))
    v = rng.normal(0, 0.3, (3, n))
    r = rng.uniform(0.003, 0.008, n)
    held = rng.uniform(0.0, 0.5, n)
    a, mom = orc.p2g_fixed_wet(c, x, v, r, held)
    a_dry, mom_dry = orc.p2g_fixed(c, x, v, r)
    frac = 4.0 / 3.0 * math.pi * r ** 3 / 0.02 ** 3
    assert abs(a.sum() - (frac * (1.0 + held)).sum() * 2.0 ** 32) <= 0.5 * n + 1e-9 * a.sum()
    assert a.sum() > a_dry.sum()
    m = orc.wet_mass(c, r, held)
    unit = 2500.0 * 0.02 ** 3
    for k in range(3):
        want = (m * v[k]).sum() / unit * 2.0 ** 32
        assert abs(mom[k].sum() - want) <= 0.5 * n + 1e-6 * abs(want)
    # heavier granules carry more momentum: the grid moves away from the dry one
    assert not np.array_equal(mom, mom_dry)


def test_held_zero_is_the_dry_path(orc):
    """held = 0 everywhere: contact forces, integrator and P2G equal the dry
    oracle functions bit for bit."""
    c = cfg()
    rng = np.random.Generator(np.random.PCG64(4))
    n = 400
    x = rng.uniform(0.03, 0.29, (3, n))
    v = rng.normal(0, 0.2, (3, n))
    r = rng.uniform(0.006, 0.012, n)
    z = np.zeros(n)
    m = orc.wet_mass(c, r, z)
    F, fa, nc = orc.contact_forces_wet(c, x, v, r, m)
    F0, fa0, nc0, _ = orc.contact_forces(c, x, v, r)
    assert nc0.sum() > 50
    assert np.array_equal(F, F0) and np.array_equal(fa, fa0) and np.array_equal(nc, nc0)
    Fd = rng.normal(0, 1e-3, (3, n))
    assert all(np.array_equal(a, b) for a, b in zip(orc.integrate_wet(c, r, m, F0, Fd, x, v),
                                                    orc.integrate(c, r, F0, Fd, x, v)))
    a, mo = orc.p2g_fixed_wet(c, x, v, r, z)
    a0, mo0 = orc.p2g_fixed(c, x, v, r)
    assert np.array_equal(a, a0) and np.array_equal(mo, mo0)
    idx = rng.choice(n, 30, replace=False)
    Fs, fs = orc.contact_forces_sample_wet(c, x, v, r, m, idx)
    assert np.array_equal(Fs, F0[:, idx]) and np.array_equal(fs, fa0[idx])


# ---- the held water's volume (Sec. 5.3) --------------------------------------

def test_lone_wet_granule_fraction_at_a_node_centre(orc):
    """A lone granule centred on a node deposits frac (1 + held) with weights
    (1/8, 3/4, 1/8) per axis and samples back alpha_s = frac (1 + held)
    sum_k w_k^2 = frac (1 + held) 0.59375^3 (each node's value rounded to
    2^-32, 27 roundings)."""
    c = cfg()
    r = np.array([0.006])
    x = np.array([[0.15], [0.17], [0.13]])  # node centres (i + 1/2) dx
    v = np.zeros((3, 1))
    frac = 4.0 / 3.0 * math.pi * 0.006 ** 3 / 0.02 ** 3
    G = int(np.prod(c["n"]))
    u = np.zeros((3, G))
    for held in (0.0, 0.25, 0.7):
        a, _ = orc.p2g_fixed_wet(c, x, v, r, np.array([held]))
        _, af = orc.g2p(c, x, u, alpha_fx=a)
        assert abs((1.0 - af[0]) - frac * (1.0 + held) * 0.59375 ** 3) <= 27 * 2.0 ** -33


@pytest.mark.parametrize("absorb_max", [0.0, 0.3])
def test_raised_clamp_of_alpha_s(orc, absorb_max):
    """A uniform solid-fraction grid alpha: G2P samples min(alpha, 0.740 (1 +
    r_max)) (partition of unity), so with r_max = 0.3 a grid at 0.9 is not
    clamped, one at 1.2 is clamped to 0.962, and a dry bed clamps both at
    0.740; the density projection's target takes the same clamp."""
    import oracle.idp as idp
    c = cfg(absorb_max=absorb_max)
    G = int(np.prod(c["n"]))
    x = np.array([[0.151, 0.2], [0.163, 0.05], [0.149, 0.31]])
    u = np.zeros((3, G))
    amax = 0.74 * (1.0 + absorb_max)
    for level in (0.9, 1.2):
        a = np.full(G, int(round(level * 2.0 ** 32)), np.int64)
        _, af = orc.g2p(c, x, u, alpha_fx=a)
        assert np.allclose(1.0 - af, min(level, amax), rtol=0, atol=2.0 ** -32)
        at = idp.target_fraction(a, 0.74, absorb_max)
        assert np.allclose(at, 1.0 - min(level, amax), rtol=0, atol=2.0 ** -32)


def test_uniform_pressure_gradient_on_a_wet_granule(orc):
    """Eq. 5a with the absorbed water counted as volume: F = -V (1 + held)
    grad p; the drag alone does not see the water (the radius is the sand's)."""
    c = cfg(c_drag=30.0)
    G = int(np.prod(c["n"]))
    gp = np.repeat(np.array([[120.0], [-35.0], [9810.0]]), G, axis=1)
    u = np.zeros((3, G))
    a0 = np.zeros(G, np.int64)
    x = np.array([[0.151], [0.163], [0.149]])
    v = np.array([[0.01], [0.0], [-0.02]])
    r = np.array([0.004])
    V = 4.0 / 3.0 * math.pi * 0.004 ** 3
    held = np.array([0.35])
    Fd = orc.fluid_forces(c, x, v, r, u, a0)
    assert np.array_equal(orc.fluid_forces(c, x, v, r, u, a0, held=held), Fd)
    F = orc.fluid_forces(dict(c, c_drag=0.0), x, v, r, u, a0, gp=gp, held=held)
    assert np.allclose(F[:, 0], -V * 1.35 * np.array([120.0, -35.0, 9810.0]), rtol=1e-14, atol=0)
    assert np.array_equal(orc.fluid_forces(c, x, v, r, u, a0, gp=gp, held=np.zeros(1)),
                          orc.fluid_forces(c, x, v, r, u, a0, gp=gp))


@pytest.mark.parametrize("held", [0.0, 0.2, 0.6])
def test_wet_sphere_released_in_still_fluid(orc, held):
    """Hydrostatic grad p = rho_0 g, virtual mass on: a wet sphere from rest
    accelerates at g V (rho_s - rho_0) / (V (rho_s + held rho_0) + rho_0 V
    (1 + held) / 2): buoyancy of the water-filled volume cancels the water's
    weight, the water's mass and added mass slow it."""
    g = np.array([0.0, 0.0, -9.81])
    c = cfg(g=list(g), vmass=1)
    G = int(np.prod(c["n"]))
    gp = np.repeat((RHO_F * g)[:, None], G, axis=1)
    u = np.zeros((3, G))
    a0 = np.zeros(G, np.int64)
    x = np.array([[0.151], [0.163], [0.149]])
    v = np.zeros((3, 1))
    r = np.array([0.004])
    H = np.array([held])
    m = orc.wet_mass(c, r, H)
    V = 4.0 / 3.0 * math.pi * 0.004 ** 3
    acc = g * V * (2500.0 - RHO_F) / (V * (2500.0 + held * RHO_F) + RHO_F * V * (1.0 + held) / 2.0)
    for k in range(1, 4):
        F = orc.fluid_forces(c, x, v, r, u, a0, gp=gp, held=H)
        x, v = orc.integrate_wet(c, r, m, np.zeros((3, 1)), F, x, v, held=H)
        assert np.allclose(v[:, 0], k * c["dt"] * acc, rtol=1e-12, atol=1e-18)


def test_wet_exchange_force_is_newtons_law(orc):
    """The exchanged force of wet granules is the whole fluid force: with the
    wet integrator's acceleration a_s, m_wet a_s = m_wet g + F_c + f_ex."""
    g = [0.0, 0.0, -9.81]
    c = cfg(g=g, vmass=1, drag_model=1, c_quad=0.5, f_unit=1e-3)
    rng = np.random.Generator(np.random.PCG64(12))
    n = 40
    x = rng.uniform(0.03, 0.29, (3, n))
    v = rng.normal(0, 0.05, (3, n))
    r = rng.uniform(0.002, 0.004, n)
    held = rng.uniform(0.0, 0.6, n)
    G = int(np.prod(c["n"]))
    u = rng.normal(0, 0.1, (3, G))
    gp = rng.normal(0, 50.0, (3, G))
    af = rng.normal(0, 0.5, (3, G))
    a0, _ = orc.p2g_fixed_wet(c, x, v, r, held)
    F = orc.fluid_forces(c, x, v, r, u, a0, gp=gp, af=af, held=held)
    Fc = rng.normal(0, 1e-4, (3, n))
    m = orc.wet_mass(c, r, held)
    _, v1 = orc.integrate_wet(c, r, m, Fc, F, x, v, held=held)
    fex = orc.exchange_force(c, r, Fc, F, held=held)
    lhs = m * (v1 - v) / c["dt"]
    rhs = m * np.array(g)[:, None] + Fc + fex
    assert np.allclose(lhs, rhs, rtol=1e-9, atol=1e-12 * np.abs(rhs).max())
    # the dry exchange of the same forces differs: the water's mass and volume matter
    assert not np.allclose(orc.exchange_force(c, r, Fc, F), fex, rtol=1e-6, atol=0)
