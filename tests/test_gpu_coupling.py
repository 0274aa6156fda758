"""GPU parity of the remaining interphase forces (Sec. 3.3 Eq. 5a-5c, Sec. 5.2
Eq. 9) and of the sand step with the exchange momentum (Alg. 2, Sec. 5.2),
through the C ABI, against the FP64 oracle on the same seeded inputs.

Bars: fluid forces to 1e-5 (FP32 form) / 1e-12 (FP64) of each granule's
force scale; the integrator with virtual mass and the exchange deposit bit
for bit (the same double arithmetic on the same inputs; the deposit is
integer); a sand step of several sub-steps to the FP32 / FP64 bars scaled by
the step's velocity change and the exchange grid's magnitude.
"""
import math

import numpy as np
import pytest

from paper_2504_00745_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-12}


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_00745_amd import gic
    gic.lib()
    import gpu_util
    return gpu_util


def bed(n=12289, seed=7, **over):
    """A thinned c2 bed (polydisperse, contacts) with seeded grad p and fluid
    acceleration fields; the coupling parameters of a sand-water mixture."""
    d = wl.make("c2", n_override=n)
    cfg = dict(d["params"], rho_f=1000.0, c_quad=0.44, f_unit=1e-4, drag_model=0, vmass=1)
    cfg.update(over)
    Gn = int(np.prod(cfg["n"]))
    rng = np.random.Generator(np.random.PCG64(seed))
    gp = np.array(cfg["g"])[:, None] * 1000.0 + rng.normal(0, 200.0, (3, Gn))
    af = rng.normal(0, 0.5, (3, Gn))
    u = d["u"] + rng.normal(0, 0.02, d["u"].shape)
    return cfg, d["x"], d["v"], d["r"], u, gp, af


def sorted_state(G, gic, cfg, x, v, r, prec):
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
    return ctx, X, V, R, ID, order, cb, ce


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("model", [0, 1])
def test_fluid_gather_matches_oracle(G, orc, prec, model):
    """Drag of either model + pressure gradient + explicit virtual-mass term
    at each granule, against the oracle; the gathered state is the input
    permuted, bit for bit."""
    import torch
    from paper_2504_00745_amd import gic
    G.say(f"[fluid gather] c2 thinned, {prec}, drag model {model}")
    cfg, x, v, r, u, gp, af = bed(drag_model=model)
    n = x.shape[1]
    ctx, X, V, R, ID, order, cb, ce = sorted_state(G, gic, cfg, x, v, r, prec)
    real = ctx.real
    Xs, Vs, Rs, IDs = torch.empty_like(X), torch.empty_like(V), torch.empty_like(R), torch.empty_like(ID)
    a0, _ = orc.p2g_fixed(cfg, x, v, r)  # P2G is order independent: the oracle's grid is the GPU's
    A0 = G.dev(a0, torch.int64)
    Ff = torch.empty(3 * n, dtype=real, device="cuda")
    gic.gic_gather_g2p_fluid(ctx, order, X.view(3, n), V, R, ID, Xs, Vs, Rs, IDs, G.dev(u.reshape(-1), real), A0,
                             cb, ce, Ff, grad_p=G.dev(gp.reshape(-1), real), acc_f=G.dev(af.reshape(-1), real))
    torch.cuda.synchronize()
    assert ctx.error() == (0, -1)
    ids = IDs.cpu().numpy()
    assert np.array_equal(Xs.view(3, n).cpu().numpy(), x[:, ids])
    assert np.array_equal(Rs.cpu().numpy(), r[ids])
    Fg = np.empty((3, n))
    Fg[:, ids] = Ff.view(3, n).double().cpu().numpy()
    Fo = orc.fluid_forces(cfg, x, v, r, u, a0, gp=gp, af=af)
    # scale: the magnitudes of the three terms, each from the oracle alone
    off = dict(cfg, c_drag=0.0, c_quad=0.0)
    Fd = orc.fluid_forces(dict(cfg, vmass=0), x, v, r, u, a0)
    Fp = orc.fluid_forces(dict(off, vmass=0), x, v, r, u, a0, gp=gp)
    Fa = orc.fluid_forces(dict(off, vmass=1), x, v, r, u, a0, af=af)
    scale = np.linalg.norm(Fd, axis=0) + np.linalg.norm(Fp, axis=0) + np.linalg.norm(Fa, axis=0) + 1e-300
    err = np.linalg.norm(Fg - Fo, axis=0)
    assert np.all(err <= TOL[prec] * scale), np.max(err / scale)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_fluid_gather_without_extra_terms_is_the_drag_gather(G, orc, prec):
    """No grad p, no fluid acceleration, linear drag: the fluid gather gives
    the drag gather's force bit for bit."""
    import torch
    from paper_2504_00745_amd import gic
    cfg, x, v, r, u, gp, af = bed(vmass=0)
    n = x.shape[1]
    ctx, X, V, R, ID, order, cb, ce = sorted_state(G, gic, cfg, x, v, r, prec)
    real = ctx.real
    a0, _ = orc.p2g_fixed(cfg, x, v, r)
    A0 = G.dev(a0, torch.int64)
    U = G.dev(u.reshape(-1), real)
    outs = []
    for fluid in (False, True):
        Xs, Vs, Rs, IDs = torch.empty_like(X), torch.empty_like(V), torch.empty_like(R), torch.empty_like(ID)
        F = torch.empty(3 * n, dtype=real, device="cuda")
        if fluid:
            gic.gic_gather_g2p_fluid(ctx, order, X.view(3, n), V, R, ID, Xs, Vs, Rs, IDs, U, A0, cb, ce, F)
        else:
            gic.gic_gather_g2p_drag(ctx, order, X.view(3, n), V, R, ID, Xs, Vs, Rs, IDs, U, A0, cb, ce, F)
        outs.append(F.cpu())
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("vmass", [0, 1])
def test_exchange_and_virtual_mass_integrate_bit_exact(G, orc, prec, vmass):
    """The exchange deposit (integer) and the virtual-mass integrator (the
    oracle's double arithmetic on the same inputs) match the oracle bit for
    bit, on the sorted state with seeded contact and fluid forces (rounded to
    the form's type on the host, the same values on both sides)."""
    import torch
    from paper_2504_00745_amd import gic
    G.say(f"[exchange + integrate] {prec}, vmass {vmass}")
    cfg, x, v, r, u, gp, af = bed(vmass=vmass, drag_model=1)
    n = x.shape[1]
    ctx, X, V, R, ID, order, cb, ce = sorted_state(G, gic, cfg, x, v, r, prec)
    real = ctx.real
    o_or = orc.stable_sort(orc.cell_keys(cfg, x))
    assert np.array_equal(order.cpu().numpy(), o_or)
    Xs, Vs, Rs, IDs = torch.empty_like(X), torch.empty_like(V), torch.empty_like(R), torch.empty_like(ID)
    gic.gic_reorder(ctx, order, X.view(3, n), V, R, ID, Xs, Vs, Rs, IDs)
    xs, vs, rs = x[:, o_or], v[:, o_or], r[o_or]
    rng = np.random.Generator(np.random.PCG64(19 + vmass))
    fc = rng.normal(0.0, 0.05, (3, n))
    ff = rng.normal(0.0, 0.01, (3, n))
    if prec == "fp32":
        fc, ff = fc.astype(np.float32).astype(np.float64), ff.astype(np.float32).astype(np.float64)
    Fc, Ff = G.dev(fc.reshape(-1), real), G.dev(ff.reshape(-1), real)
    FS = torch.zeros(3 * ctx.G, dtype=torch.int64, device="cuda")
    gic.gic_exchange_p2g(ctx, Xs.view(3, n), Rs, Fc, Ff, cb, ce, 0.25, FS)
    X1, V1 = Xs.clone(), Vs.clone()
    A1 = torch.empty(ctx.G, dtype=torch.int64, device="cuda")
    M1 = torch.empty(3 * ctx.G, dtype=torch.int64, device="cuda")
    gic.gic_integrate_p2g(ctx, X1.view(3, n), V1, Rs, Fc, Ff, cb, ce, A1, M1)
    torch.cuda.synchronize()
    assert ctx.error() == (0, -1)
    fs_o = orc.exchange_p2g(cfg, xs, rs, fc, ff, 0.25)
    assert np.array_equal(FS.view(3, -1).cpu().numpy(), fs_o)
    assert np.abs(fs_o).max() > 2 ** 32  # the deposit is not trivially zero
    x1o, v1o = orc.integrate_vm(cfg, rs, fc, ff, xs, vs)
    x1g, v1g = X1.view(3, n).cpu().numpy(), V1.view(3, n).cpu().numpy()
    if vmass:  # the virtual-mass update is written in the oracle's operation order
        assert np.array_equal(v1g, v1o) and np.array_equal(x1g, x1o)
        a1o, m1o = orc.p2g_fixed(cfg, x1o, v1o, rs)
        assert np.array_equal(A1.cpu().numpy(), a1o) and np.array_equal(M1.view(3, -1).cpu().numpy(), m1o)
    else:  # the plain update multiplies by 1/m where the oracle divides by m
        assert np.allclose(v1g, v1o, rtol=1e-14, atol=1e-18) and np.allclose(x1g, x1o, rtol=1e-15, atol=0)
        a0, _ = orc.p2g_fixed(cfg, x, v, r)
        assert int(A1.sum().item()) == int(a0.sum())  # the total does not depend on positions


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_sand_step_matches_oracle(G, orc, prec):
    """A sand step of ceil(3.5) = 4 sub-steps with frozen grad p and fluid
    acceleration, virtual mass and quadratic drag: sub-step count, final
    positions and velocities and the exchange grid against the oracle's sand
    step."""
    import torch
    from paper_2504_00745_amd import gic
    G.say(f"[sand step] c2 thinned, {prec}")
    cfg, x, v, r, u, gp, af = bed(drag_model=1)
    n = x.shape[1]
    sim = gic.Simulator(cfg, x, v, r, u, prec, r_max=float(r.max()))
    real = sim.ctx.real
    a0, _ = orc.p2g_fixed(cfg, x, v, r)
    assert np.array_equal(sim.alpha.cpu().numpy(), a0)
    FS = torch.zeros(3 * sim.ctx.G, dtype=torch.int64, device="cuda")
    Dt = 3.5 * cfg["dt"]
    N = sim.sand_step(Dt, grad_p=G.dev(gp.reshape(-1), real), acc_f=G.dev(af.reshape(-1), real), fs=FS)
    torch.cuda.synchronize()
    assert sim.ctx.error() == (0, -1)
    out = orc.sand_step(cfg, Dt, x, v, r, u, a0, gp=gp, af=af)
    assert N == out["N"] == 4
    xg, vg = sim.state_in_input_order()
    dv = np.linalg.norm(out["v"] - v, axis=0)
    tol = TOL[prec] * (dv.max() + 1e-300)
    assert np.max(np.linalg.norm(vg - out["v"], axis=0)) <= tol
    assert np.max(np.linalg.norm(xg - out["x"], axis=0)) <= Dt * tol + 1e-15
    fsg = FS.view(3, -1).cpu().numpy().astype(np.float64)
    fso = out["fs"].astype(np.float64)
    assert np.max(np.abs(fsg - fso)) <= TOL[prec] * np.abs(fso).max() + 4.0 * N


def test_sand_step_of_one_substep_is_gic_step(G, orc):
    """With the drag-only coupling and Dt = dt the sand step is gic_step, bit
    for bit (same kernels, the fluid gather reducing to the drag gather)."""
    import torch
    from paper_2504_00745_amd import gic
    cfg, x, v, r, u, gp, af = bed(vmass=0)
    sims = [gic.Simulator(cfg, x, v, r, u, "fp32", r_max=float(r.max())) for _ in range(2)]
    sims[0].step()
    assert sims[1].sand_step(cfg["dt"]) == 1
    torch.cuda.synchronize()
    for k in ("x", "v", "r", "id"):
        assert torch.equal(sims[0].cur[k], sims[1].cur[k])
    assert torch.equal(sims[0].alpha, sims[1].alpha) and torch.equal(sims[0].mom, sims[1].mom)
