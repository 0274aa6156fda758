"""GPU parity of the wet-granule integrator and momentum deposit (Sec. 5.3,
Eq. 19: m = V (rho_s + held rho_f)) through gic_integrate_p2g_wet, against the
oracle's wet integrator and wet P2G on the same sorted state and seeded
forces (rounded to the form's type on the host).

Bars: with virtual mass the update follows the oracle's operation order and
the state and both int64 grids are bit-exact; without it the update
multiplies by 1/m where the oracle divides (states within 1e-14), and the
grids are compared through their position-independent fraction total; held
= 0 gives gic_integrate_p2g bit for bit.
"""
import numpy as np
import pytest

from paper_2504_00745_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_00745_amd import gic
    gic.lib()
    import gpu_util
    return gpu_util


def sorted_bed(G, gic, cfg, x, v, r, prec):
    import torch
    n = x.shape[1]
    ctx = gic.Context(cfg, n, prec, r_max=float(r.max()))
    X, V, R = G.dev(x.reshape(-1)), G.dev(v.reshape(-1)), G.dev(r)
    ID = torch.arange(n, dtype=torch.int32, device="cuda")
    key = torch.empty(n, dtype=torch.int32, device="cuda")
    order = torch.empty(n, dtype=torch.int32, device="cuda")
    cb = torch.empty(ctx.K, dtype=torch.int32, device="cuda")
    ce = torch.empty(ctx.K, dtype=torch.int32, device="cuda")
    gic.gic_sort_cells(ctx, X.view(3, n), key, order, cb, ce)
    Xs, Vs, Rs, IDs = torch.empty_like(X), torch.empty_like(V), torch.empty_like(R), torch.empty_like(ID)
    gic.gic_reorder(ctx, order, X.view(3, n), V, R, ID, Xs, Vs, Rs, IDs)
    return ctx, Xs, Vs, Rs, order, cb, ce


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("vmass", [0, 1])
def test_wet_integrate_p2g_matches_oracle(G, orc, prec, vmass):
    import torch
    from paper_2504_00745_amd import gic
    G.say(f"[wet integrate + P2G] {prec}, vmass {vmass}")
    d = wl.make("c2", n_override=12289)
    cfg = dict(d["params"], rho_f=1000.0, vmass=vmass)
    x, v, r = d["x"], d["v"], d["r"]
    n = x.shape[1]
    ctx, Xs, Vs, Rs, order, cb, ce = sorted_bed(G, gic, cfg, x, v, r, prec)
    o_or = orc.stable_sort(orc.cell_keys(cfg, x))
    assert np.array_equal(order.cpu().numpy(), o_or)
    xs, vs, rs = x[:, o_or], v[:, o_or], r[o_or]
    rng = np.random.Generator(np.random.PCG64(41 + vmass))
    held = rng.uniform(0.0, 0.5, n)
    fc = rng.normal(0.0, 0.05, (3, n))
    fd = rng.normal(0.0, 0.01, (3, n))
    if prec == "fp32":
        fc, fd = fc.astype(np.float32).astype(np.float64), fd.astype(np.float32).astype(np.float64)
    Fc, Fd = G.dev(fc.reshape(-1), ctx.real), G.dev(fd.reshape(-1), ctx.real)
    H = G.dev(held)
    X1, V1 = Xs.clone(), Vs.clone()
    A1 = torch.empty(ctx.G, dtype=torch.int64, device="cuda")
    M1 = torch.empty(3 * ctx.G, dtype=torch.int64, device="cuda")
    gic.gic_integrate_p2g_wet(ctx, X1.view(3, n), V1, Rs, H, Fc, Fd, cb, ce, A1, M1)
    torch.cuda.synchronize()
    assert ctx.error() == (0, -1)
    m = orc.wet_mass(cfg, rs, held)
    x1o, v1o = orc.integrate_wet(cfg, rs, m, fc, fd, xs, vs)
    x1g, v1g = X1.view(3, n).cpu().numpy(), V1.view(3, n).cpu().numpy()
    if vmass:
        assert np.array_equal(v1g, v1o) and np.array_equal(x1g, x1o)
        a1o, m1o = orc.p2g_fixed_wet(cfg, x1o, v1o, rs, held)
        assert np.array_equal(A1.cpu().numpy(), a1o) and np.array_equal(M1.view(3, -1).cpu().numpy(), m1o)
    else:
        assert np.allclose(v1g, v1o, rtol=1e-14, atol=1e-18) and np.allclose(x1g, x1o, rtol=1e-15, atol=0)
        a0, _ = orc.p2g_fixed(cfg, x, v, r)
        assert int(A1.sum().item()) == int(a0.sum())
    # the wet velocities differ from the dry update: the water's mass matters
    X2, V2 = Xs.clone(), Vs.clone()
    A2 = torch.empty_like(A1)
    M2 = torch.empty_like(M1)
    gic.gic_integrate_p2g(ctx, X2.view(3, n), V2, Rs, Fc, Fd, cb, ce, A2, M2)
    assert not torch.equal(V1, V2)
    # held = 0: the dry entry point's state and grids bit for bit
    X3, V3 = Xs.clone(), Vs.clone()
    A3 = torch.empty_like(A1)
    M3 = torch.empty_like(M1)
    gic.gic_integrate_p2g_wet(ctx, X3.view(3, n), V3, Rs, torch.zeros_like(H), Fc, Fd, cb, ce, A3, M3)
    torch.cuda.synchronize()
    assert torch.equal(X3, X2) and torch.equal(V3, V2) and torch.equal(A3, A2) and torch.equal(M3, M2)


def test_wet_entry_needs_held(G):
    import torch
    from paper_2504_00745_amd import gic
    d = wl.make("c2", n_override=2000)
    n = d["x"].shape[1]
    ctx, Xs, Vs, Rs, order, cb, ce = sorted_bed(G, gic, d["params"], d["x"], d["v"], d["r"], "fp32")
    F = torch.zeros(3 * n, dtype=torch.float32, device="cuda")
    A = torch.empty(ctx.G, dtype=torch.int64, device="cuda")
    M = torch.empty(3 * ctx.G, dtype=torch.int64, device="cuda")
    rc = gic.lib().gic_integrate_p2g_wet(ctx.handle, n, gic._ptr(Xs), gic._ptr(Vs), gic._ptr(Rs), None, gic._ptr(F),
                                         gic._ptr(F), gic._ptr(cb), gic._ptr(ce), gic._ptr(A), gic._ptr(M), 0, None)
    assert rc == 1
