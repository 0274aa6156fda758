"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars: bit-exact keys, order, cell ranges, touching pairs (the production
contact kernel's own pair output) and int64 P2G grids on identical inputs;
forces, velocities and positions within 1e-5 (FP32 form) or 1e-12 (plain
FP64 form) of the scale of the terms that sum into them, per granule and per
step from an identical state:
    |F - F_or| <= tol S,  S = sum_j |F_ij| + |F_wall| (oracle)
    |v - v_or| <= tol (|v_or| + dt (S + |F_d| + m |g|) / m)
because a dense bed's net force cancels to far below its terms.  The
sampled fluid velocity per component within tol sum_k w_k |u_k| (the
granule's own stencil sum of magnitudes, which bounds the rounding of the
27-term sum), the fluid fraction within tol (a volume fraction), the drag
within tol beta (|u_at| + |v|).
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


def _cases():
    return ["c1", "c1b", "c4s", "c2s"]


def _make(name):
    if name == "c4s":
        d = wl.make("c4", n_override=12289)   # ragged: 6 sort tiles + a tail
    elif name == "c2s":
        d = wl.make("c2", n_override=30001)
    else:
        d = wl.make(name)
    return d


def _rmax(name, r):
    return float(r.max())


def _check_sort(orc, d, out):
    cfg = d["params"]
    key = orc.cell_keys(cfg, d["x"])
    assert np.array_equal(out["key"], key)
    order = orc.stable_sort(key)
    assert np.array_equal(out["order"], order)
    assert np.array_equal(out["ids"], order)
    b, e = orc.cell_ranges(cfg, key, order)
    assert np.array_equal(out["cell_begin"], b)
    assert np.array_equal(out["cell_end"], e)


def _force_scale(orc, d, Fd=None):
    cfg = d["params"]
    F, fa, nc, ns = orc.contact_forces(cfg, d["x"], d["v"], d["r"])
    return F, fa, nc, ns


def _check_step(G, orc, d, out, prec, name):
    cfg = d["params"]
    tol = TOL[prec]
    x, v, r, u = d["x"], d["v"], d["r"], d["u"]
    # identical alpha grid on both sides (the GPU's own initial P2G, itself
    # checked bit-exact against the oracle below)
    a0_or, _ = orc.p2g_fixed(cfg, x, v, r)
    assert np.array_equal(out["alpha0"], a0_or), "initial P2G alpha differs"
    st = orc.step(cfg, x, v, r, u, a0_or)
    Fc, fa, nc, ns = orc.contact_forces(cfg, x, v, r)
    assert np.array_equal(out["ncont"], nc), "contact counts differ"
    # G2P, drag, per granule
    uabs, _ = orc.g2p(cfg, x, np.abs(u), alpha_fx=a0_or)  # sum_k w_k |u_k| per component
    assert np.all(np.abs(out["u_at"] - st["u_at"]) <= tol * uabs + 1e-300), \
        np.max(np.abs(out["u_at"] - st["u_at"]) / (uabs + 1e-300))
    assert np.abs(out["alpha_f"] - st["alpha_f"]).max() <= tol
    m = cfg["rho_s"] * (((4.0 * math.pi / 3.0) * r) * r) * r
    fdn = np.linalg.norm(st["Fd"], axis=0)
    beta = cfg["c_drag"] * 6 * math.pi * cfg["eta_f"] * r
    dscale = beta * (np.linalg.norm(st["u_at"], axis=0) + np.linalg.norm(v, axis=0))
    assert np.all(np.linalg.norm(out["Fd"] - st["Fd"], axis=0) <= tol * dscale + 1e-300)
    # contact force
    err = np.linalg.norm(out["Fc"] - Fc, axis=0)
    assert np.all(err <= tol * fa + 1e-300), f"{name}: max contact err/scale {np.max(err / (fa + 1e-300))}"
    # velocities and positions
    g = np.linalg.norm(cfg["g"])
    S = fa + fdn + tol * dscale + m * g
    vscale = np.linalg.norm(st["v"], axis=0) + cfg["dt"] * S / m
    verr = np.linalg.norm(out["v1"] - st["v"], axis=0)
    assert np.all(verr <= tol * vscale), f"{name}: max v err/scale {np.max(verr / vscale)}"
    xerr = np.linalg.norm(out["x1"] - st["x"], axis=0)
    ulp = 4 * np.spacing(np.abs(st["x"]).max(axis=0))
    assert np.all(xerr <= cfg["dt"] * tol * vscale + ulp)
    # P2G after the move: the total fraction does not depend on positions, so
    # the advanced grid holds the oracle's total exactly; and P2G of the
    # oracle's advanced state through the HIP path equals the oracle's P2G
    # of it bit for bit
    assert int(out["alpha1"].sum()) == int(a0_or.sum())
    a1g, m1g = G.p2g_of(cfg, st["x"], st["v"], r, prec, r_max=_rmax(name, r))
    a1, m1 = orc.p2g_fixed(cfg, st["x"], st["v"], r)
    assert np.array_equal(a1g, a1)
    assert np.array_equal(m1g, m1)
    return nc.sum(), ns.sum()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", _cases())
def test_stage_parity(G, orc, name, prec):
    G.say(f"[parity] {name} {prec}")
    d = _make(name)
    out = G.run_stages(d["params"], d["x"], d["v"], d["r"], d["u"], prec, r_max=_rmax(name, d["r"]))
    _check_sort(orc, d, out)
    nct, nsl = _check_step(G, orc, d, out, prec, name)
    assert out["err"] == (0, -1)
    if name in ("c1b", "c4s", "c2s"):
        assert nct > 0
    G.say(f"[parity] {name} {prec} ok: contacts {nct} sliding {nsl}")


@pytest.mark.parametrize("name", ["c1b", "c4s", "c2s"])
def test_contact_pairs_bit_exact(G, orc, name):
    """The touching pairs that the production contact kernel sums (its pair
    output) equal the oracle's cell-list pair set, itself pinned to the
    O(N^2) definition; both forms run the same double test."""
    G.say(f"[pairs] {name}")
    d = _make(name)
    x, r = d["x"], d["r"]
    for prec in ("fp32", "fp64"):
        out = G.run_stages(d["params"], x, d["v"], r, d["u"], prec, r_max=float(r.max()))
        ref = set(map(tuple, np.sort(orc.pairs_cells(d["params"], x, r), 1).tolist()))
        assert out["pairs"] == ref and len(ref) > 0


def test_contact_pairs_at_the_contact_distance(G, orc):
    """Pairs placed within a few ulps of d = r_i + r_j, along random
    directions, across cell faces and with unequal radii: the single-precision
    candidate filter with margin M must keep every one that the exact double
    test keeps; the pair output equals the O(N^2) definition."""
    G.say("[pairs] at the contact distance")
    d = wl.make("c1", n_override=1)
    cfg = d["params"]
    rng = np.random.Generator(np.random.PCG64(31))
    xs, rs = [], []
    L = cfg["n"][0] * cfg["dx"]
    for k in range(1500):
        ri, rj = rng.uniform(0.004, 0.01), rng.uniform(0.004, 0.01)
        c = rng.uniform(0.03, L - 0.03, 3)
        if k % 3 == 0:  # centre the pair on a cell face
            c[k % 2] = np.round(c[k % 2] / cfg["cell"]) * cfg["cell"]
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        dd = (ri + rj) * (1.0 + rng.integers(-6, 7) * 2.0 ** -52)
        xs += [c - 0.5 * dd * u, c + 0.5 * dd * u]
        rs += [ri, rj]
    x = np.array(xs).T.copy()
    r = np.array(rs)
    # keep pairs apart from each other: drop any granule that touches a granule of another pair
    ref_all = orc.pairs_brute(x, r)
    bad = set()
    for i, j in ref_all:
        if i // 2 != j // 2:
            bad |= {i // 2, j // 2}
    keep = np.array([k for k in range(x.shape[1]) if k // 2 not in bad])
    x, r = np.ascontiguousarray(x[:, keep]), r[keep]
    v = np.zeros_like(x)
    ref = set(map(tuple, np.sort(orc.pairs_brute(x, r), 1).tolist()))
    assert 100 < len(ref) < x.shape[1] // 2  # touching and non-touching pairs both occur
    for prec in ("fp32", "fp64"):
        out = G.run_stages(cfg, x, v, r, np.zeros_like(d["u"]), prec, r_max=0.01)
        assert out["pairs"] == ref
        assert out["err"] == (0, -1)


@pytest.mark.parametrize("n", [0, 1, 2, 2047, 2048, 2049])
def test_sort_edge_sizes(G, orc, n):
    G.say(f"[sort] n={n}")
    d = wl.make("c2", n_override=max(n, 1))
    x, v, r = d["x"][:, :n], d["v"][:, :n], d["r"][:n]
    out = G.run_stages(d["params"], x, v, r, d["u"], "fp32", r_max=0.01)
    if n:
        _check_sort(orc, dict(d, x=x), out)
    else:
        assert not out["cell_begin"].any() and not out["cell_end"].any()
    assert out["err"] == (0, -1)


def test_sort_many_equal_keys_stable(G, orc):
    """All granules in a handful of cells: long runs of equal keys keep input
    order across tiles and passes."""
    G.say("[sort] equal keys")
    d = wl.make("c2", n_override=20000)
    rng = np.random.Generator(np.random.PCG64(1))
    cells = rng.integers(0, 5, 20000)
    x = np.stack([0.005 + cells * 0.02, np.full(20000, 0.005), np.full(20000, 0.5)])
    out = G.run_stages(d["params"], x, d["v"], np.full(20000, 0.004), d["u"], "fp32", r_max=0.01)
    _check_sort(orc, dict(d, x=x), out)


def test_latched_errors(G, orc):
    """Non-finite and out-of-box positions and oversized radii latch the
    documented code and the first offending index."""
    G.say("[errors]")
    d = wl.make("c1")
    x = d["x"].copy()
    x[1, 17] = np.nan
    out = G.run_stages(d["params"], x, d["v"], d["r"], d["u"], "fp64", r_max=0.01)
    assert out["err"][0] == 5
    x = d["x"].copy()
    x[2, 33] = -0.01
    out = G.run_stages(d["params"], x, d["v"], d["r"], d["u"], "fp64", r_max=0.01)
    assert out["err"] == (4, 33)
    r = d["r"].copy()
    r[5] = 0.011
    out = G.run_stages(d["params"], d["x"], d["v"], r, d["u"], "fp64", r_max=0.01)
    assert out["err"][0] == 6


@pytest.mark.parametrize("name,vscale", [("c4s", 1.0), ("c4s", 1e4), ("c2s", 1.0), ("c1", 1.0)])
def test_whole_step_matches_stages(G, name, vscale):
    """gic_step (grids assembled from stored brick tiles) runs the same
    arithmetic as the staged sequence (grids cleared, tiles added with
    atomics): bit-identical state, grids and order, for cells of 1.6, 2 and
    1 node spacings.  With the velocities scaled by 1e4 (up to two nodes per
    step) many granules leave their brick's tile after the move and are
    deposited by the escape pass."""
    import torch
    from paper_2504_00745_amd import gic
    G.say(f"[step] {name} fp32, v x {vscale}")
    d = _make(name)
    n = d["x"].shape[1]
    d["v"] = d["v"] * vscale
    rm = _rmax(name, d["r"])
    out = G.run_stages(d["params"], d["x"], d["v"], d["r"], d["u"], "fp32", r_max=rm)
    sim = gic.Simulator(d["params"], d["x"].reshape(3, n), d["v"].reshape(3, n), d["r"], d["u"].reshape(-1),
                        "fp32", r_max=rm)
    # the Simulator starts from its own sorted copy; feed the stage run the same
    # alpha grid and compare state by input index
    assert np.array_equal(sim.alpha.cpu().numpy(), out["alpha0"])
    sim.step()
    x1, v1 = sim.state_in_input_order()
    assert np.array_equal(x1, out["x1"])
    assert np.array_equal(v1, out["v1"])
    assert np.array_equal(sim.alpha.cpu().numpy(), out["alpha1"])
    assert np.array_equal(sim.mom.cpu().numpy().reshape(3, -1), out["mom1"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_contact_dense_brick_and_many_partners(G, orc, prec):
    """Rare paths of the contact kernel: a brick whose one-cell shell holds
    more granules than fit in LDS (global candidate path), and granules with
    more touching partners than the per-granule list (second candidate
    walk).  Forces and contact counts still match the oracle."""
    G.say(f"[contact rare paths] {prec}")
    d = wl.make("c2", n_override=1000)
    cfg = d["params"]
    rng = np.random.Generator(np.random.PCG64(21))
    # 3000 small granules packed in one 0.08 m brick (cell 0.02): shell overflow
    xs = rng.uniform(0.405, 0.475, (3, 3000))
    rs = np.full(3000, 0.0018)
    # big granules each ringed by 30 small touching ones: long partner lists
    big = []
    for c in ([0.9, 0.9, 0.9], [0.3, 1.0, 0.6]):
        c = np.array(c)
        u = rng.normal(size=(30, 3))
        u /= np.linalg.norm(u, axis=1)[:, None]
        big.append(np.concatenate([c[None, :], c + u * (0.0099 + 0.0029)], 0))
    xb = np.concatenate(big, 0).T
    rb = np.tile(np.concatenate([[0.0099], np.full(30, 0.003)]), 2)
    x = np.concatenate([xs, xb], 1)
    r = np.concatenate([rs, rb])
    v = rng.normal(0, 0.05, x.shape)
    n = x.shape[1]
    u = np.zeros((3, int(np.prod(cfg["n"]))))
    out = G.run_stages(cfg, x, v, r, u, prec, r_max=0.0099)
    Fc, fa, nc, ns = orc.contact_forces(cfg, x, v, r)
    assert nc.max() >= 20 and nc[:3000].sum() > 3000  # shell overflow and long lists both occur
    assert np.array_equal(out["ncont"], nc)
    err = np.linalg.norm(out["Fc"] - Fc, axis=0)
    assert np.all(err <= TOL[prec] * fa + 1e-300), np.max(err / (fa + 1e-300))
    assert out["err"] == (0, -1)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fused_stages_match_separate(G, prec):
    """gic_gather_g2p_drag = reorder + G2P + drag and gic_integrate_p2g =
    integrate + P2G, bit for bit (state, sampled fluid values, forces, int64
    grids), on a polydisperse bed with a ragged tail; accumulate=1 adds to
    the grids."""
    import torch
    from paper_2504_00745_amd import gic
    G.say(f"[fused stages] c2s {prec}")
    d = _make("c2s")
    cfg, x, v, r, u = d["params"], d["x"], d["v"], d["r"], d["u"]
    n = x.shape[1]
    ctx = gic.Context(cfg, n, prec, float(r.max()))
    real = ctx.real
    X, V, R = G.dev(x.reshape(-1)), G.dev(v.reshape(-1)), G.dev(r)
    ID = torch.arange(n, dtype=torch.int32, device="cuda")
    key = torch.empty(n, dtype=torch.int32, device="cuda")
    order = torch.empty(n, dtype=torch.int32, device="cuda")
    cb = torch.empty(ctx.K, dtype=torch.int32, device="cuda")
    ce = torch.empty(ctx.K, dtype=torch.int32, device="cuda")
    gic.gic_sort_cells(ctx, X.view(3, n), key, order, cb, ce)
    e = lambda like: torch.empty_like(like)
    Xs, Vs, Rs, IDs = e(X), e(V), e(R), e(ID)
    gic.gic_reorder(ctx, order, X.view(3, n), V, R, ID, Xs, Vs, Rs, IDs)
    U = G.dev(u.reshape(-1), real)
    A0 = torch.zeros(ctx.G, dtype=torch.int64, device="cuda")
    gic.gic_p2g(ctx, Xs.view(3, n), Vs, Rs, cb, ce, A0, None)
    uat = torch.empty(3 * n, dtype=real, device="cuda")
    af = torch.empty(n, dtype=real, device="cuda")
    gic.gic_g2p(ctx, Xs.view(3, n), U, A0, None, uat, af)
    Fd = torch.empty(3 * n, dtype=real, device="cuda")
    gic.gic_drag(ctx, Rs, Vs, uat, af, Fd)
    Fc = torch.empty(3 * n, dtype=real, device="cuda")
    gic.gic_contact_forces(ctx, Xs.view(3, n), Vs, Rs, cb, ce, Fc)
    X1, V1 = Xs.clone(), Vs.clone()
    gic.gic_integrate(ctx, Rs, Fc, Fd, X1, V1)
    A1 = torch.empty(ctx.G, dtype=torch.int64, device="cuda")
    M1 = torch.empty(3 * ctx.G, dtype=torch.int64, device="cuda")
    gic.gic_p2g(ctx, X1.view(3, n), V1, Rs, cb, ce, A1, M1)
    # fused
    X2, V2, R2, ID2 = e(X), e(V), e(R), e(ID)
    Fd2, uat2, af2 = e(Fd), e(uat), e(af)
    gic.gic_gather_g2p_drag(ctx, order, X.view(3, n), V, R, ID, X2, V2, R2, ID2, U, A0, cb, ce, Fd2, uat2, af2)
    for a, b in ((X2, Xs), (V2, Vs), (R2, Rs), (ID2, IDs), (Fd2, Fd), (uat2, uat), (af2, af)):
        assert torch.equal(a, b)
    Fd3 = e(Fd)
    gic.gic_gather_g2p_drag(ctx, order, X.view(3, n), V, R, None, X2, V2, R2, None, U, A0, cb, ce, Fd3)
    assert torch.equal(Fd3, Fd)
    A2 = torch.full((ctx.G,), 7, dtype=torch.int64, device="cuda")
    M2 = torch.full((3 * ctx.G,), 7, dtype=torch.int64, device="cuda")
    X3, V3 = X2.clone(), V2.clone()
    gic.gic_integrate_p2g(ctx, X2.view(3, n), V2, R2, Fc, Fd2, cb, ce, A2, M2)
    assert torch.equal(X2, X1) and torch.equal(V2, V1)
    assert torch.equal(A2, A1) and torch.equal(M2, M1)
    gic.gic_integrate_p2g(ctx, X3.view(3, n), V3, R2, Fc, Fd2, cb, ce, A2, M2, accumulate=True)
    assert torch.equal(A2, 2 * A1) and torch.equal(M2, 2 * M1)
    assert ctx.error() == (0, -1)


@pytest.mark.parametrize("moved", [0, 1, 37, 4096, 4097, 20000])
def test_sort_incremental_path(G, orc, moved):
    """A second sort on the same context, of the gathered state with some
    granules moved to other cells, takes the incremental path while at most
    4096 keys changed and the radix passes beyond; keys, order and cell
    ranges are bit-exact against the oracle either way.  A third sort, of an
    unrelated bed with the same count, still sorts exactly."""
    import torch
    from paper_2504_00745_amd import gic
    G.say(f"[sort incremental] moved {moved}")
    d = wl.make("c2", n_override=30001)
    cfg, x, r = d["params"], d["x"], d["r"]
    n = x.shape[1]
    ctx = gic.Context(cfg, n, "fp32", float(r.max()))
    key = torch.empty(n, dtype=torch.int32, device="cuda")
    order = torch.empty(n, dtype=torch.int32, device="cuda")
    cb = torch.empty(ctx.K, dtype=torch.int32, device="cuda")
    ce = torch.empty(ctx.K, dtype=torch.int32, device="cuda")

    def sort_and_check(xx):
        X = G.dev(xx.reshape(-1))
        gic.gic_sort_cells(ctx, X.view(3, n), key, order, cb, ce)
        torch.cuda.synchronize()
        k_or = orc.cell_keys(cfg, xx)
        o_or = orc.stable_sort(k_or)
        assert np.array_equal(key.cpu().numpy().view(np.uint32), k_or)
        assert np.array_equal(order.cpu().numpy(), o_or)
        b_or, e_or = orc.cell_ranges(cfg, k_or, o_or)
        assert np.array_equal(cb.cpu().numpy(), b_or)
        assert np.array_equal(ce.cpu().numpy(), e_or)
        return o_or

    o1 = sort_and_check(x)
    xs = np.ascontiguousarray(x[:, o1])  # the gathered state of the first sort
    rng = np.random.Generator(np.random.PCG64(100 + moved))
    idx = rng.choice(n, moved, replace=False)
    L = np.array([cfg["n"][a] * cfg["dx"] for a in range(3)])
    xs[:, idx] = rng.uniform(0.0, 1.0, (3, moved)) * L[:, None] * 0.999
    sort_and_check(xs)
    other = wl.make("c2", n_override=30001, seed=77)["x"]
    sort_and_check(other)
    assert ctx.error() == (0, -1)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_kept_brick_list_gives_the_same_bits(G, prec):
    """gic_brick_list: brick kernels that reuse the kept schedule (fixed and
    unquantised P2G, contact with and without the pair output, the fused
    gather) give the bits of the same calls building their own, on a
    polydisperse bed with a ragged tail; a new sort drops the kept list."""
    import torch
    from paper_2504_00745_amd import gic
    G.say(f"[kept brick list] c2s {prec}")
    d = _make("c2s")
    cfg, x, v, r, u = d["params"], d["x"], d["v"], d["r"], d["u"]
    n = x.shape[1]
    X, V, R = G.dev(x.reshape(-1)), G.dev(v.reshape(-1)), G.dev(r)
    ID = torch.arange(n, dtype=torch.int32, device="cuda")

    def run(keep):
        ctx = gic.Context(cfg, n, prec, float(r.max()))
        real = ctx.real
        key = torch.empty(n, dtype=torch.int32, device="cuda")
        order = torch.empty(n, dtype=torch.int32, device="cuda")
        cb = torch.empty(ctx.K, dtype=torch.int32, device="cuda")
        ce = torch.empty(ctx.K, dtype=torch.int32, device="cuda")
        gic.gic_sort_cells(ctx, X.view(3, n), key, order, cb, ce)
        if keep:
            gic.gic_brick_list(ctx, cb, ce)
        e = lambda like: torch.empty_like(like)
        Xs, Vs, Rs, IDs = e(X), e(V), e(R), e(ID)
        gic.gic_reorder(ctx, order, X.view(3, n), V, R, ID, Xs, Vs, Rs, IDs)
        A = torch.zeros(ctx.G, dtype=torch.int64, device="cuda")
        M = torch.zeros(3 * ctx.G, dtype=torch.int64, device="cuda")
        gic.gic_p2g(ctx, Xs.view(3, n), Vs, Rs, cb, ce, A, M)
        Fc = torch.empty(3 * n, dtype=real, device="cuda")
        gic.gic_contact_forces(ctx, Xs.view(3, n), Vs, Rs, cb, ce, Fc)
        Fc2 = torch.empty(3 * n, dtype=real, device="cuda")
        P = torch.empty(8 * n, dtype=torch.int32, device="cuda")
        gic.gic_contact_forces(ctx, Xs.view(3, n), Vs, Rs, cb, ce, Fc2, pair_ids=P)
        U = G.dev(u.reshape(-1), real)
        X2, V2, R2, ID2 = e(X), e(V), e(R), e(ID)
        Fd = torch.empty(3 * n, dtype=real, device="cuda")
        gic.gic_gather_g2p_drag(ctx, order, X.view(3, n), V, R, ID, X2, V2, R2, ID2, U, A, cb, ce, Fd)
        out = [A, M, Fc, Fc2, P, Fd, X2]
        if prec == "fp64":
            Ar = torch.empty(ctx.G, dtype=torch.float64, device="cuda")
            Mr = torch.empty(3 * ctx.G, dtype=torch.float64, device="cuda")
            gic.gic_p2g_real(ctx, Xs.view(3, n), Vs, Rs, cb, ce, Ar, Mr)
            out += [Ar, Mr]
        # a new sort of other positions drops the kept list: these calls
        # then build the list of the new tables
        Xb = X.clone()
        Xb.view(3, n)[0] += 0.37 * cfg["cell"]
        Xb.view(3, n)[0].clamp_(max=cfg["n"][0] * cfg["dx"] * 0.999)
        gic.gic_sort_cells(ctx, Xb.view(3, n), key, order, cb, ce)
        Xbs, Vbs, Rbs = e(X), e(V), e(R)
        gic.gic_reorder(ctx, order, Xb.view(3, n), V, R, None, Xbs, Vbs, Rbs, None)
        Ab = torch.zeros(ctx.G, dtype=torch.int64, device="cuda")
        gic.gic_p2g(ctx, Xbs.view(3, n), Vbs, Rbs, cb, ce, Ab, None)
        out.append(Ab)
        torch.cuda.synchronize()
        assert ctx.error() == (0, -1)
        return out

    for a, b in zip(run(True), run(False)):
        assert torch.equal(a, b)


def test_stage_times_cover_the_step(G):
    """gic_stage_timing / gic_stage_times: seven stages per step (sort,
    gather, contact, exchange, grid clear, integrate + P2G, assembly) over
    the steps asked for; on a bed whose grids are assembled from brick tiles
    the assembly takes time, while the exchange deposit (none in gic_step)
    and the grid clear (none when the grids are assembled) are only the gap
    between two adjacent events (a few microseconds); the stages sum to at
    most the steps' own elapsed time."""
    import torch
    from paper_2504_00745_amd import gic
    G.say("[stage times] c4s fp32")
    d = _make("c4s")
    n = d["x"].shape[1]
    sim = gic.Simulator(d["params"], d["x"].reshape(3, n), d["v"].reshape(3, n), d["r"], d["u"].reshape(-1),
                        "fp32", r_max=_rmax("c4s", d["r"]))
    sim.step()
    torch.cuda.synchronize()
    sim.ctx.stage_timing(8)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(4):
        sim.step()
    e1.record()
    ms, k = sim.ctx.stage_times()
    sim.ctx.stage_timing(0)
    assert k == 4
    assert list(ms) == list(gic.Context.STAGES) and len(ms) == 7
    assert all(v >= 0.0 for v in ms.values())
    assert ms["assemble"] > 0.0 and ms["integrate_p2g"] > 0.0 and ms["sort"] > 0.0
    assert ms["exchange"] / k < 0.010 and ms["grid_clear"] / k < 0.010  # ms per step
    assert sum(ms.values()) <= 1.05 * e0.elapsed_time(e1)
    assert sim.ctx.error() == (0, -1)


def _contact_direct(gic, ctx, x, v, r):
    """Sort, reorder and the direct contact kernel (no pair output) on ctx;
    forces and counts in input order."""
    import torch
    n = x.shape[1]
    X, V, R = G_dev(x.reshape(-1)), G_dev(v.reshape(-1)), G_dev(r)
    ID = torch.arange(n, dtype=torch.int32, device="cuda")
    key = torch.empty(n, dtype=torch.int32, device="cuda")
    order = torch.empty(n, dtype=torch.int32, device="cuda")
    cb = torch.empty(ctx.K, dtype=torch.int32, device="cuda")
    ce = torch.empty(ctx.K, dtype=torch.int32, device="cuda")
    gic.gic_sort_cells(ctx, X.view(3, n), key, order, cb, ce)
    Xs, Vs, Rs, IDs = torch.empty_like(X), torch.empty_like(V), torch.empty_like(R), torch.empty_like(ID)
    gic.gic_reorder(ctx, order, X.view(3, n), V, R, ID, Xs, Vs, Rs, IDs)
    F = torch.empty(3 * n, dtype=ctx.real, device="cuda")
    nc = torch.empty(n, dtype=torch.int32, device="cuda")
    gic.gic_contact_forces(ctx, Xs.view(3, n), Vs, Rs, cb, ce, F, nc)
    torch.cuda.synchronize()  # (the context's record of the largest shell has landed too)
    ids = IDs.cpu().numpy()
    Fi = np.empty((3, n))
    Fi[:, ids] = F.view(3, n).cpu().numpy()
    nci = np.empty(n, dtype=np.int32)
    nci[ids] = nc.cpu().numpy()
    return Fi, nci


def G_dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", torch.float64).contiguous()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_contact_shell_array_sized_from_earlier_calls(G, prec):
    """The direct contact kernel sizes its LDS shell array from the largest
    brick shell that an earlier call on the context recorded (the record of
    every 16th call reaches the host).  After calls on a sparse bed (a small
    array), a bed with one dense brick (its shell beyond that array, within
    the largest) takes the global candidate path for that brick and gives
    the bits of a fresh context (largest array, LDS path); once the dense
    bed's record has reached the host (the 17th call on the context), the
    calls size for it and give the same bits again."""
    from paper_2504_00745_amd import gic
    G.say(f"[contact shell size] {prec}")
    d = wl.make("c2", n_override=20000)
    cfg = d["params"]
    rng = np.random.Generator(np.random.PCG64(33))
    # 700 small granules in a 0.04 m cube inside one 0.08 m brick (cell 0.02)
    xs = rng.uniform(0.42, 0.46, (3, 700))
    x = np.concatenate([d["x"], xs], 1)
    r = np.concatenate([d["r"], np.full(700, 0.0018)])
    v = np.concatenate([d["v"], rng.normal(0, 0.05, (3, 700))], 1)
    rm = float(d["r"].max())
    ctx = gic.Context(cfg, x.shape[1], prec, rm)
    for _ in range(3):  # the sparse bed: the record settles on its shells
        _contact_direct(gic, ctx, d["x"], d["v"], d["r"])
    ref = _contact_direct(gic, gic.Context(cfg, x.shape[1], prec, rm), x, v, r)
    for k in range(17):  # calls 3 .. 19 on ctx: call 16 copies the dense record
        F, nc = _contact_direct(gic, ctx, x, v, r)
        assert np.array_equal(F, ref[0]), k
        assert np.array_equal(nc, ref[1]), k
    assert ref[1][-700:].sum() > 700  # the dense brick's granules touch
    assert ctx.error() == (0, -1)
