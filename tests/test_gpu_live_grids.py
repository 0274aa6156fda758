"""The stepping path's grids after each step are the P2G of the state it
left, node for node, while the path rewrites only the 4-node segments that a
stencil reaches now or reached at the previous step (the rest of the grids
hold that step's zeros): a bed that drifts through the box leaves zeros
behind it; granules that leave their brick's tile (deposited by the escape
pass) mark their nodes; a caller's write into the grids between steps is
undone by the next step once gic_set_params is called, or when the write
came from a call on the context.

Bar: bit-identical alpha and momentum grids against gic_p2g of the same state
on a context of its own (grids cleared, every granule deposited)."""
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


def _drifting_bed(nodes_per_step=0.5):
    """The thinned c4 bed (a layer of four nodes on the floor of the box,
    wall to wall) with a common drift upwards added to its velocities."""
    d = wl.make("c4", n_override=12289)
    p = d["params"]
    v = d["v"].copy()
    v[2] += nodes_per_step * p["dx"] / p["dt"]
    return d, v


def _reference(gic, ref, sim):
    """gic_p2g of the simulator's current state on the context ref."""
    import torch
    s = sim.scratch
    A = torch.empty_like(sim.alpha)
    M = torch.empty_like(sim.mom)
    gic.gic_p2g(ref, sim.cur["x"], sim.cur["v"], sim.cur["r"], s["cell_begin"], s["cell_end"], A, M)
    return A, M


def _check(gic, ref, sim, what):
    import torch
    A, M = _reference(gic, ref, sim)
    assert torch.equal(sim.alpha, A), what
    assert torch.equal(sim.mom, M), what
    assert int((A != 0).sum()) > 0


def test_grids_follow_a_drifting_bed(G):
    """Twelve steps of a bed that drifts by six nodes: every step's grids
    are the full P2G of its state, including the zeros the bed left."""
    import torch
    from paper_2504_00745_amd import gic
    G.say("[live grids] drifting bed")
    d, v = _drifting_bed()
    n = d["x"].shape[1]
    rm = float(d["r"].max())
    sim = gic.Simulator(d["params"], d["x"], v, d["r"], d["u"], "fp32", r_max=rm)
    ref = gic.Context(d["params"], n, "fp32", rm)
    A0 = sim.alpha.clone()
    for k in range(12):
        sim.step()
        _check(gic, ref, sim, f"step {k}")
    # the bed moved: nodes that held granules at the start are zero now
    left = (A0 != 0) & (sim.alpha == 0)
    assert int(left.sum()) > 0
    assert sim.ctx.error() == (0, -1)


def test_escaped_granules_mark_their_nodes(G):
    """A drift of 3 nodes per step (more than a tile's slack of at most two
    nodes): the granules leave their brick's tile after the move and are
    deposited by the escape pass; the steps after still rewrite (and clear)
    the nodes they reached."""
    from paper_2504_00745_amd import gic
    G.say("[live grids] escapes")
    d, v = _drifting_bed(3.0)
    n = d["x"].shape[1]
    rm = float(d["r"].max())
    sim = gic.Simulator(d["params"], d["x"], v, d["r"], d["u"], "fp32", r_max=rm)
    ref = gic.Context(d["params"], n, "fp32", rm)
    for k in range(6):
        sim.step()
        _check(gic, ref, sim, f"step {k}")
    assert sim.ctx.error() == (0, -1)


def test_writes_into_the_grids_between_steps(G):
    """A caller's value written into an empty region of the momentum grid is
    cleared by the next step after gic_set_params; a gic_p2g on the context
    into the simulator's grids (of a state moved elsewhere) is noticed
    without it."""
    import torch
    from paper_2504_00745_amd import gic
    G.say("[live grids] writes between steps")
    d, v = _drifting_bed()
    n = d["x"].shape[1]
    rm = float(d["r"].max())
    sim = gic.Simulator(d["params"], d["x"], v, d["r"], d["u"], "fp32", r_max=rm)
    ref = gic.Context(d["params"], n, "fp32", rm)
    for _ in range(2):
        sim.step()
    far = sim.mom.numel() - 1  # the last node of the z component: the box's top corner
    assert int(sim.mom[far]) == 0
    sim.mom[far] = 12345
    sim.ctx.set_params()
    sim.step()
    _check(gic, ref, sim, "after set_params")
    assert int(sim.mom[far]) == 0
    # the state lifted to the top of the box, deposited into the simulator's
    # grids by a call on its context, then a step from the true state
    # (grouped by the cells of the true state: granules outside their brick's
    # tile take the global path, so the deposit is still every granule's)
    s = sim.scratch
    x_up = sim.cur["x"].clone().view(3, n)
    L2 = d["params"]["n"][2] * d["params"]["dx"]
    x_up[2] += 0.5 * L2
    gic.gic_p2g(sim.ctx, x_up, sim.cur["v"], sim.cur["r"], s["cell_begin"], s["cell_end"], sim.alpha, sim.mom)
    up = sim.alpha != 0
    sim.step()
    _check(gic, ref, sim, "after a P2G of another state")
    assert int((up & (sim.alpha == 0)).sum()) > 0
    assert sim.ctx.error() == (0, -1)
