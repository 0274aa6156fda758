"""Seeded synthetic granular beds and fluid fields.

This module only generates inputs: granule positions, velocities and radii,
a fluid velocity on the grid nodes, and the parameter block.  It holds none of
the method's arithmetic (no contact, transfer, drag or integration), so both
the GPU path and the CPU oracle may draw their inputs from it.

The paper's own scenes are bespoke and not available; these beds stand in for
them with the sizes, radius laws and packings named for each workload.  Every
random draw comes from numpy's PCG64 seeded with the workload's seed.

Workloads (granules N, grid, neighbour cell edge h):
  c1      4,096 r=0.01 on a jittered 16^3 lattice at solid fraction 0.40 in a
          0.64^3 box, v ~ N(0, 0.05^2), 32^3 grid dx=0.02, 8 Fourier modes
          A=0.1, no gravity, dt=1e-5, plain FP64.  No pair touches.
  c1b     as c1 but lattice spacing 0.02(1-1e-3), jitter 1e-6: every lattice
          neighbour overlaps by ~2e-5 m (contact parity case).
  c2      262,144 log-normal radii (median 0.005, sigma 0.2, clipped to
          [0.003, 0.01]) by random sequential addition at solid fraction 0.30
          over the full x-y footprint, 128^3 grid dx=0.01, h=0.02, gravity,
          16 modes A=0.2, dt=5e-6, 100 steps.
  c3      4,194,304 r=0.001 on a 128x256x128 simple-cubic lattice of spacing
          2r-1e-8 (every face neighbour in contact) filling x<0.256, z<0.256
          of a 256x128x128 grid dx=0.004 (dam-break column), v=0, u=0,
          gravity, dt=2e-6, 50 steps, h=dx.
  c4      65,536 bidisperse r=0.004/0.006 (70/30 by count) by random
          sequential addition at 0.30 in z<0.245, v ~ N(0,0.05^2), 64^3 grid
          dx=0.01, h=0.016, 8 modes A=0.1, C_d=1000, dt=1e-5, 20 steps.
  c3s     the c3 bed scaled down for tests: 8,192 granules on a 16x32x16
          lattice in a 32^3 grid, the same spacing, jitter, cell and step.
  c5      16,777,216 radii U[0.00075, 0.0015] on a jittered 512x256x128
          lattice of spacing 0.003 (lower half of a 512x256x256 grid,
          dx=0.003, h=dx), v ~ N(0, 0.02^2), shear u_x = 0.5 z/L_z plus 32
          modes A=0.05, gravity, dt=1e-6, 20 steps.

Random sequential addition places spheres at radius r/1.01 and then uses the
true radius, so light contacts (overlap <= 1% of r) exist from the first step.
"""
import math

import numpy as np

# Material parameters shared by every workload (kg, m, s).
_BASE = dict(kn=1.0e5, restitution=0.5, kt_ratio=1.0, mu=0.5, rho_s=2500.0, eta_f=1.0e-3, c_drag=1.0,
             alpha_max=0.740, walls=0x3F)

WORKLOADS = ("c1", "c1b", "c2", "c3", "c3s", "c4", "c5")


def _params(n, dx, cell, dt, g, **kw):
    n = [int(a) for a in n]
    L = [a * dx for a in n]
    nc = [max(1, int(math.floor(La / cell * (1 + 1e-12)))) for La in L]
    p = dict(_BASE)
    p.update(n=n, dx=float(dx), nc=nc, cell=float(cell), dt=float(dt), g=[float(a) for a in g])
    p.update(kw)
    return p


def spec(name: str) -> dict:
    """Parameter block and recipe of a workload (no arrays)."""
    G0 = [0.0, 0.0, -9.81]
    Z = [0.0, 0.0, 0.0]
    if name in ("c1", "c1b"):
        p = _params([32] * 3, 0.02, 0.02, 1e-5, Z)
        return dict(name=name, N=4096, steps=1, precision="fp64", params=p, seed=1 if name == "c1" else 11)
    if name == "c2":
        p = _params([128] * 3, 0.01, 0.02, 5e-6, G0)
        return dict(name=name, N=262144, steps=100, precision="fp32", params=p, seed=2)
    if name == "c3":
        p = _params([256, 128, 128], 0.004, 0.004, 2e-6, G0)
        return dict(name=name, N=4194304, steps=50, precision="fp32", params=p, seed=3)
    if name == "c3s":
        p = _params([32, 32, 32], 0.004, 0.004, 2e-6, G0)
        return dict(name=name, N=8192, steps=50, precision="fp32", params=p, seed=3)
    if name == "c4":
        p = _params([64] * 3, 0.01, 0.016, 1e-5, Z, c_drag=1000.0)
        return dict(name=name, N=65536, steps=20, precision="fp64", params=p, seed=4, checkpoint=5)
    if name == "c5":
        p = _params([512, 256, 256], 0.003, 0.003, 1e-6, G0)
        return dict(name=name, N=16777216, steps=20, precision="fp32", params=p, seed=5)
    raise KeyError(name)


# ---------------------------------------------------------------------------
# Fluid velocity on the nodes
# ---------------------------------------------------------------------------

def fourier_field(n, dx, modes, amp, rng, shear=0.0):
    """Divergence-free sum of `modes` sine modes sampled at the cell-centred
    nodes (i+1/2) dx; returns (3, G) float64, x-fastest.

    u(x) = A/sqrt(M) sum_m a_m sin(2 pi k_m . (x/L) + phi_m) with integer
    wave vectors k_m in {-3..3}^3 \\ {0}, unit amplitudes a_m orthogonal to
    k_m/L and phases uniform in [0, 2 pi); optional shear adds s z/L_z to u_x.
    """
    nx, ny, nz = (int(a) for a in n)
    L = np.array([nx * dx, ny * dx, nz * dx])
    u = np.zeros((3, nz, ny, nx))
    if modes:
        k = rng.integers(-3, 4, size=(modes, 3))
        for m in range(modes):
            while not k[m].any():
                k[m] = rng.integers(-3, 4, size=3)
        q = k / L
        a = rng.standard_normal((modes, 3))
        a -= (np.sum(a * q, 1) / np.sum(q * q, 1))[:, None] * q
        a /= np.linalg.norm(a, axis=1)[:, None]
        phi = rng.uniform(0.0, 2.0 * np.pi, modes)
        xs = [(np.arange(na) + 0.5) * dx for na in (nx, ny, nz)]
        for m in range(modes):
            ex = np.exp(2j * np.pi * q[m, 0] * xs[0])
            ey = np.exp(2j * np.pi * q[m, 1] * xs[1])
            ez = np.exp(2j * np.pi * q[m, 2] * xs[2]) * np.exp(1j * phi[m])
            for kz in range(nz):
                s = np.imag(ez[kz] * np.outer(ey, ex))
                for c in range(3):
                    u[c, kz] += (amp / math.sqrt(modes)) * a[m, c] * s
    if shear:
        zc = (np.arange(nz) + 0.5) * dx
        u[0] += (shear * zc / L[2])[:, None, None]
    return u.reshape(3, -1)


# ---------------------------------------------------------------------------
# Placement
# ---------------------------------------------------------------------------

def _lattice(counts, spacing, origin, jitter, rng):
    cx, cy, cz = counts
    gz, gy, gx = np.meshgrid(np.arange(cz), np.arange(cy), np.arange(cx), indexing="ij")
    pos = np.stack([gx.ravel(), gy.ravel(), gz.ravel()]).astype(np.float64)
    pos = (pos + 0.5) * spacing + np.asarray(origin, np.float64)[:, None]
    if np.isscalar(jitter):
        if jitter:
            pos += rng.uniform(-jitter, jitter, size=pos.shape)
    else:
        pos += rng.uniform(-1.0, 1.0, size=pos.shape) * jitter[None, :]
    return pos


_RSA = None


def _rsa_lib():
    """The random-sequential-addition helper (csrc/rsa.c), built on first use."""
    global _RSA
    if _RSA is None:
        import ctypes as C
        import os
        import subprocess
        here = os.path.dirname(os.path.abspath(__file__))
        so = os.path.join(here, "libgicrsa.so")
        src = os.path.join(here, "csrc", "rsa.c")
        if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
            subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-o", so + ".tmp", src, "-lm"], check=True)
            os.replace(so + ".tmp", so)
        L = C.CDLL(so)
        D = C.POINTER(C.c_double)
        L.rsa_place.restype = C.c_double
        L.rsa_place.argtypes = [C.c_int64, D, D, D, C.c_double, C.c_uint64, C.c_int32, C.c_double, D]
        _RSA = L
    return _RSA


def rsa(radii, box_lo, box_hi, rng, zcap=None, max_attempts=2000, grow=0.05):
    """Random sequential addition of spheres with the given radii inside
    [box_lo, box_hi], in index order; a sphere that finds no room after
    max_attempts tries raises the box top by grow*diameter.  Returns
    ((3, N) positions, final box top)."""
    import ctypes as C
    radii = np.ascontiguousarray(radii, np.float64)
    N = radii.shape[0]
    lo = np.ascontiguousarray(box_lo, np.float64)
    hi = np.ascontiguousarray(box_hi, np.float64)
    zcap = float(hi[2] * 2.0 if zcap is None else zcap)
    pos = np.zeros((3, N))
    seed = int(rng.integers(0, 2 ** 63))
    D = C.POINTER(C.c_double)
    top = _rsa_lib().rsa_place(N, radii.ctypes.data_as(D), lo.ctypes.data_as(D), hi.ctypes.data_as(D), zcap, seed,
                               int(max_attempts), float(grow), pos.ctypes.data_as(D))
    if top < 0:
        raise RuntimeError("random sequential addition found no room below the height cap")
    return pos, top


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def make(name: str, seed=None, n_override=None) -> dict:
    """Arrays and parameters of a workload.

    Returns dict(x (3,N) f64, v (3,N) f64, r (N,) f64, u (3,G) f64,
    params, steps, precision, name).  n_override shrinks c2/c4-type beds
    (fewer granules, same law) for quick tests.
    """
    s = spec(name)
    p = s["params"]
    rng = np.random.Generator(np.random.PCG64(s["seed"] if seed is None else seed))
    n, dx = p["n"], p["dx"]
    L = np.array([a * dx for a in n])
    if name in ("c1", "c1b"):
        r0 = 0.01
        if name == "c1":
            sp = ((4.0 / 3.0) * math.pi * r0 ** 3 / 0.40) ** (1.0 / 3.0)
            jit = 0.0009
        else:
            sp = 0.02 * (1.0 - 1e-3)
            jit = 1e-6
        side = 16 * sp
        x = _lattice((16, 16, 16), sp, (L - side) / 2.0, jit, rng)
        N = x.shape[1]
        r = np.full(N, r0)
        v = rng.normal(0.0, 0.05, size=(3, N))
        u = fourier_field(n, dx, 8, 0.1, rng)
    elif name in ("c2", "c4"):
        N = s["N"] if n_override is None else int(n_override)
        if name == "c2":
            r = np.clip(0.005 * np.exp(0.2 * rng.standard_normal(N)), 0.003, 0.01)
        else:
            r = np.where(rng.random(N) < 0.7, 0.004, 0.006)
        vol = float(np.sum((4.0 / 3.0) * math.pi * r ** 3))
        H = vol / (0.30 * L[0] * L[1])
        # largest spheres first (denser random packing), then a random input order
        big_first = np.argsort(-r, kind="stable")
        xs, _ = rsa(r[big_first] / 1.01, [0.0, 0.0, 0.0], [L[0], L[1], H], rng, zcap=L[2])
        x = np.empty_like(xs)
        x[:, big_first] = xs
        perm = rng.permutation(N)
        x, r = x[:, perm], r[perm]
        if name == "c2":
            v = np.zeros((3, N))
            u = fourier_field(n, dx, 16, 0.2, rng)
        else:
            v = rng.normal(0.0, 0.05, size=(3, N))
            u = fourier_field(n, dx, 8, 0.1, rng)
    elif name in ("c3", "c3s"):
        r0 = 0.001
        sp = 2 * r0 - 1e-8
        x = _lattice((128, 256, 128) if name == "c3" else (16, 32, 16), sp, (0.0, 0.0, 0.0), 2e-9, rng)
        N = x.shape[1]
        r = np.full(N, r0)
        v = np.zeros((3, N))
        u = np.zeros((3, int(np.prod(n))))
    elif name == "c5":
        sp = 0.003
        counts = (512, 256, 128)
        N = int(np.prod(counts))
        r = rng.uniform(0.00075, 0.0015, N)
        jit = np.maximum(sp / 2.0 - r / 1.01, 0.0)
        gz, gy, gx = np.meshgrid(np.arange(counts[2]), np.arange(counts[1]), np.arange(counts[0]), indexing="ij")
        x = np.stack([gx.ravel(), gy.ravel(), gz.ravel()]).astype(np.float64)
        del gx, gy, gz
        x = (x + 0.5) * sp
        x += rng.uniform(-1.0, 1.0, size=x.shape) * jit[None, :]
        v = rng.normal(0.0, 0.02, size=(3, N))
        u = fourier_field(n, dx, 32, 0.05, rng, shear=0.5)
    else:
        raise KeyError(name)
    return dict(name=name, x=np.ascontiguousarray(x), v=np.ascontiguousarray(v), r=np.ascontiguousarray(r),
                u=np.ascontiguousarray(u), params=p, steps=s["steps"], precision=s["precision"])



# ---------------------------------------------------------------------------
# Density-projection inputs (Sec. 5.1): a sand fraction grid in int64 fixed
# point (what the P2G of a bed gives), the fluid particles' own fraction and
# the cell labels (0 fluid, 1 air, 2 solid), seeded and synthetic.
# ---------------------------------------------------------------------------

IDP_CASES = ("p1", "p2", "c3")


def idp_case(name: str, seed=None) -> dict:
    """p1: 32^3 cells dx = 0.02; p2: a ragged 23 x 17 x 29 grid; c3: the
    dam-break grid (256 x 128 x 128, dx = 0.004) with the sand column of the
    c3 bed (x < 0.256 m, z < 0.256 m, solid fraction pi/6).  Each: fluid up
    to 3/4 of the height and air above, a submerged solid block, the sand
    fraction of the column (or blob) with +-0.01 noise, and the fluid
    particles' fraction = (1 - sand fraction)(1 + 0.08 f) with f a smooth
    seeded field of unit amplitude, compressed 1.8-fold in a ball (beyond the
    1.5 clamp of the ratio)."""
    if name == "p1":
        n, dx, s0 = (32, 32, 32), 0.02, 11
    elif name == "p2":
        n, dx, s0 = (23, 17, 29), 0.02, 12
    elif name == "c3":
        n, dx, s0 = (256, 128, 128), 0.004, 13
    else:
        raise KeyError(name)
    rng = np.random.Generator(np.random.PCG64(s0 if seed is None else seed))
    nx, ny, nz = n
    zc, yc, xc = np.meshgrid(*[(np.arange(m) + 0.5) * dx for m in (nz, ny, nx)], indexing="ij")
    L = np.array([nx, ny, nz]) * dx
    if name == "c3":
        sand = np.where((xc < 0.256) & (zc < 0.256), math.pi / 6.0, 0.0)
    else:
        c = np.array([0.3, 0.5, 0.35]) * L
        blob = np.exp(-(((xc - c[0]) ** 2 + (yc - c[1]) ** 2 + (zc - c[2]) ** 2) / (2 * (0.2 * L.min()) ** 2)))
        sand = 0.62 * blob + np.where(xc < 0.2 * L[0], 0.55, 0.0)
    sand = np.clip(sand + rng.uniform(-0.01, 0.01, sand.shape) * (sand > 0), 0.0, 0.95)
    alpha_fx = np.rint(sand * 2.0 ** 32).astype(np.int64)
    f = fourier_field(n, dx, 8, 1.0, rng)[0].reshape(nz, ny, nx)
    f /= max(np.abs(f).max(), 1e-300)
    astar = (1.0 - sand) * (1.0 + 0.08 * f)
    cb = np.array([0.7, 0.4, 0.3]) * L
    ball = (xc - cb[0]) ** 2 + (yc - cb[1]) ** 2 + (zc - cb[2]) ** 2 < (0.1 * L.min()) ** 2
    astar = np.where(ball, 1.8 * astar, astar)
    label = np.zeros((nz, ny, nx), np.uint8)
    label[int(round(0.75 * nz)):] = 1
    label[: nz // 3, ny // 3: ny // 2, int(0.6 * nx): int(0.75 * nx)] = 2
    p = _params(n, dx, dx, 1e-4, (0.0, 0.0, -9.81))
    return dict(name=name, params=p, alpha_fx=alpha_fx.reshape(-1), alpha_star=astar.reshape(-1),
                label=label.reshape(-1), shape=(nz, ny, nx))
