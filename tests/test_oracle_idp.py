"""Pins of the oracle's density projection (Sec. 5.1, Eq. 12b, Eq. 13; App. B
discretisation): discrete eigenmodes of the constant-coefficient operator
under Dirichlet (air) and Neumann (solid) faces, the exact solution of a
layered variable-coefficient column by flux integration, two independent
forms of the operator, symmetry and definiteness, the displacement moving
exactly the excess fluid out of every cell, and the two clamps."""
import math

import numpy as np
import pytest

FL, AIR, SOL = 0, 1, 2


def air_shell(m):
    """Fluid interior of shape m (nz, ny, nx) inside a one-cell layer of air."""
    lab = np.full(tuple(k + 2 for k in m), AIR, np.uint8)
    lab[1:-1, 1:-1, 1:-1] = FL
    return lab


def test_dirichlet_box_eigenmode(orc):
    """All-air surroundings, constant alpha_f' = c: L = c (-Laplacian_h) with
    zero boundary values, whose eigenvectors are products of
    sin(pi k (i + 1) / (m + 1)) with eigenvalue c sum 2 (1 - cos(pi k / (m + 1)))."""
    I = orc.idp
    m = (5, 7, 9)  # nz, ny, nx: distinct, so a transposed axis fails
    lab = air_shell(m)
    c = 0.6
    at = np.full(lab.shape, c)
    k = (2, 3, 4)
    modes = [np.sin(math.pi * k[a] * np.arange(1, m[a] + 1) / (m[a] + 1)) for a in range(3)]
    v = np.zeros(lab.shape)
    v[1:-1, 1:-1, 1:-1] = modes[0][:, None, None] * modes[1][None, :, None] * modes[2][None, None, :]
    lam = c * sum(2 * (1 - math.cos(math.pi * k[a] / (m[a] + 1))) for a in range(3))
    Lv = I.apply(at, lab, v)
    assert np.allclose(Lv[lab == FL], lam * v[lab == FL], rtol=0, atol=1e-13)
    q = I.solve(at, lab, lam * v)
    assert np.allclose(q, v, rtol=0, atol=1e-12)


def test_neumann_walls_and_free_surface_eigenmode(orc):
    """Solid walls on the sides and bottom (the box boundary) and air on top:
    cosine modes cos(pi k (i + 1/2) / m) across the walls and, vertically,
    cos(pi (k + 1/2) (i + 1/2) / (m + 1/2)) (zero slope at the floor, zero at
    the air cell's centre), eigenvalue c sum 2 (1 - cos theta)."""
    I = orc.idp
    mz, my, mx = 6, 5, 8
    lab = np.full((mz + 1, my, mx), FL, np.uint8)
    lab[-1] = AIR
    c = 0.45
    at = np.full(lab.shape, c)
    kx, ky, kz = 3, 1, 2
    tx, ty, tz = math.pi * kx / mx, math.pi * ky / my, math.pi * (kz + 0.5) / (mz + 0.5)
    vx = np.cos(tx * (np.arange(mx) + 0.5))
    vy = np.cos(ty * (np.arange(my) + 0.5))
    vz = np.cos(tz * (np.arange(mz) + 0.5))
    v = np.zeros(lab.shape)
    v[:-1] = vz[:, None, None] * vy[None, :, None] * vx[None, None, :]
    lam = c * sum(2 * (1 - math.cos(t)) for t in (tx, ty, tz))
    Lv = I.apply(at, lab, v)
    assert np.allclose(Lv[lab == FL], lam * v[lab == FL], rtol=0, atol=1e-13)
    q = I.solve(at, lab, lam * v)
    assert np.allclose(q, v, rtol=0, atol=1e-12)


def test_layered_column_by_flux_integration(orc):
    """A column whose alpha_f' varies with height only, walls on the sides
    and floor, air on top: the flux through face i + 1/2 is the sum of the
    right-hand side below it, so q_i = sum_{k >= i} F_{k+1/2} / beta_{k+1/2}
    with beta the arithmetic mean of the two cells' alpha_f' (App. B) and the
    air cell's own alpha_f' on the top face."""
    I = orc.idp
    rng = np.random.Generator(np.random.PCG64(2))
    m, ny, nx = 12, 3, 4
    az = rng.uniform(0.26, 1.0, m + 1)
    s1 = rng.normal(0, 0.1, m)
    lab = np.full((m + 1, ny, nx), FL, np.uint8)
    lab[-1] = AIR
    at = np.broadcast_to(az[:, None, None], lab.shape).copy()
    s = np.zeros(lab.shape)
    s[:-1] = s1[:, None, None]
    q = I.solve(at, lab, s)
    F = np.cumsum(s1)                     # F_{i+1/2}, i = 0..m-1
    beta = 0.5 * (az[:-1] + az[1:])       # beta_{i+1/2}
    qz = np.cumsum((F / beta)[::-1])[::-1]
    assert np.allclose(q[:-1], qz[:, None, None], rtol=1e-12, atol=1e-15)
    assert not q[-1].any()


def test_operator_forms_agree_symmetric_positive(orc):
    """The slicing form of L and the assembled sparse matrix give the same
    product on a random labelled grid; the matrix is symmetric and
    <q, L q> > 0 for q nonzero on the fluid (air present)."""
    I = orc.idp
    rng = np.random.Generator(np.random.PCG64(4))
    shape = (7, 9, 11)
    lab = rng.choice([FL, AIR, SOL], size=shape, p=[0.75, 0.15, 0.10]).astype(np.uint8)
    at = rng.uniform(0.26, 1.0, shape)
    q = rng.normal(0, 1, shape)
    A = I.matrix(at, lab)
    assert np.allclose(I.apply(at, lab, q).ravel(), A @ q.ravel(), rtol=1e-13, atol=1e-14)
    assert abs(A - A.T).max() == 0
    qf = np.where(lab == FL, q, 0.0)
    assert float(qf.ravel() @ (A @ qf.ravel())) > 0
    d = I.diagonal(at, lab)
    assert np.array_equal(d.ravel(), A.diagonal())


def test_displacement_moves_the_excess_fluid(orc):
    """With neither clamp active, the fluid the face displacements carry out
    of each fluid cell, sum over faces of beta d_out / dx, equals its excess
    alpha_f* - alpha_f' (the linearised fraction after the move is the
    target): the projection of Eq. 12b-13 does what it is for."""
    I = orc.idp
    rng = np.random.Generator(np.random.PCG64(5))
    shape = (8, 6, 10)
    lab = np.full(shape, FL, np.uint8)
    lab[-2:] = AIR
    lab[2:4, 2:4, 3:6] = SOL
    at = rng.uniform(0.3, 1.0, shape)
    ast = at * (1 + rng.uniform(-0.2, 0.2, shape))
    dx = 0.01
    s = I.rhs(at, ast, lab)
    q = I.solve(at, lab, s)
    fx, fy, fz = I.displacement(q, lab, dx)
    assert max(np.abs(f).max() for f in (fx, fy, fz)) < dx  # clamp inactive
    out = np.zeros(shape)
    for axis, f in ((2, fx), (1, fy), (0, fz)):
        lab_j = np.full(shape, SOL, np.uint8)
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        n = shape[axis]
        sl_lo[axis] = slice(0, n - 1)
        sl_hi[axis] = slice(1, n)
        at_j = np.zeros(shape)
        at_j[tuple(sl_lo)] = at[tuple(sl_hi)]
        at_m = np.zeros(shape)
        at_m[tuple(sl_hi)] = at[tuple(sl_lo)]
        up = [slice(None)] * 3
        lo = [slice(None)] * 3
        up[axis] = slice(1, n + 1)
        lo[axis] = slice(0, n)
        out += 0.5 * (at + at_j) * f[tuple(up)] / dx    # through the + face, outward along +axis
        out -= 0.5 * (at + at_m) * f[tuple(lo)] / dx    # through the - face, outward along -axis
    fl = lab == FL
    assert np.allclose(out[fl], (ast - at)[fl], rtol=1e-9, atol=1e-13)


def test_clamps(orc):
    """The fraction ratio is clamped to [0.5, 1.5] and a face displacement to
    one cell width; the target fraction is 1 - min(alpha 2^-32, 0.740)."""
    I = orc.idp
    at = np.array([[[0.5, 0.5, 0.5, 0.5]]])
    lab = np.zeros(at.shape, np.uint8)
    s = I.rhs(at, np.array([[[0.1, 0.2, 1.0, 0.6]]]), lab)
    assert np.array_equal(s, [[[0.5 * -0.5, 0.5 * -0.5, 0.5 * 0.5, 0.5 * (1.2 - 1)]]])
    q = np.array([[[3.0, 0.0, -0.2, 0.0]]])
    fx, fy, fz = I.displacement(q, lab, 0.5)
    assert np.array_equal(fx[0, 0], [0.0, 0.5, 0.1, -0.1, 0.0])
    a = np.array([0, 1 << 31, 3 << 30, 1 << 32, 5 << 32])
    assert np.array_equal(I.target_fraction(a, 0.74), [1.0, 0.5, 0.26, 0.26, 0.26])
