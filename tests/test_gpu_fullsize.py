"""Parity at full workload sizes, in the launch configuration bench.py times
(one gic_step of the Simulator, FP32 form):

  c3: 4,194,304 granules, 256x128x128 grid (the benchmark workload)
  c5: 16,777,216 granules, 512x256x256 grid (the largest)

Checked: cell keys, sort order and cell ranges bit-exact against the oracle
over all granules; the int64 P2G grids of the input state bit-exact against
the oracle over the whole grid, and the advanced grid's total (independent
of positions) equal to it; contact forces and advanced velocities of a
random sample of granules against the oracle (computed one by one: contact,
G2P and drag of the input state), to the 1e-5 FP32-form bar of the
pair-force sums; the touching partners of the sampled granules from the
contact kernel's pair output equal the oracle's; at c3, the HIP P2G of the
oracle's whole advanced state equals the oracle's P2G of it bit for bit.
"""
import math

import numpy as np
import pytest

from paper_2504_00745_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_00745_amd import gic
    gic.lib()
    import gpu_util
    return gpu_util


@pytest.mark.parametrize("name", ["c3", "c5"])
def test_full_size_step(T, orc, name):
    import torch
    from paper_2504_00745_amd import gic
    T.say(f"[full size] {name}: generating")
    d = wl.make(name)
    cfg, x, v, r, u = d["params"], d["x"], d["v"], d["r"], d["u"]
    n = x.shape[1]
    T.say(f"[full size] {name}: {n} granules, GPU step")
    sim = gic.Simulator(cfg, x, v, r, u, "fp32", r_max=float(r.max()))
    # the Simulator's state is the sorted copy of the input: id[q] = input index
    ids0 = sim.cur["id"].cpu().numpy()
    # P2G of the input state (the Simulator's initial grids), whole grid
    T.say(f"[full size] {name}: oracle P2G")
    a0, m0 = orc.p2g_fixed(cfg, x, v, r)
    assert np.array_equal(sim.alpha.cpu().numpy(), a0)
    assert np.array_equal(sim.mom.cpu().numpy().reshape(3, -1), m0)
    del m0
    sim.step()
    torch.cuda.synchronize()
    assert sim.ctx.error() == (0, -1)
    s = sim.scratch
    # sort of the step: keys of the (sorted) state, stable order, ranges
    x_in = x[:, ids0]
    key = orc.cell_keys(cfg, x_in)
    T.say(f"[full size] {name}: oracle sort")
    order = orc.stable_sort(key)
    assert np.array_equal(s["key"][:n].cpu().numpy().view(np.uint32), key)
    assert np.array_equal(s["order"][:n].cpu().numpy(), order)
    b, e = orc.cell_ranges(cfg, key, order)
    assert np.array_equal(s["cell_begin"].cpu().numpy(), b)
    assert np.array_equal(s["cell_end"].cpu().numpy(), e)
    del b, e, key
    # the advanced grid's total fraction does not depend on positions
    x1, v1 = sim.state_in_input_order()
    assert int(sim.alpha.sum().item()) == int(a0.sum())
    # sampled contact forces and velocities
    rng = np.random.Generator(np.random.PCG64(7))
    idx = rng.choice(n, 3000, replace=False)
    Fs, fa = orc.contact_forces_sample(cfg, x, v, r, idx)
    pos = np.empty(n, np.int64)
    pos[ids0[order]] = np.arange(n)  # input index -> sorted position of the step
    Fg = s["f_contact"].view(3, n).double().cpu().numpy()[:, pos[idx]]
    err = np.linalg.norm(Fg - Fs, axis=0)
    assert np.all(err <= 1e-5 * fa + 1e-300), np.max(err / (fa + 1e-300))
    m = cfg["rho_s"] * (((4.0 * math.pi / 3.0) * r[idx]) * r[idx]) * r[idx]
    uat, af = orc.g2p(cfg, x[:, idx], u, alpha_fx=a0)
    Fd = orc.drag(cfg, r[idx], v[:, idx], uat, af)
    g = np.array(cfg["g"])[:, None]
    v_pred = v[:, idx] + cfg["dt"] * ((Fs + Fd) / m + g)
    scale = np.linalg.norm(v_pred, axis=0) + cfg["dt"] * (fa + np.linalg.norm(Fd, axis=0) + m * 9.81) / m
    assert np.all(np.linalg.norm(v1[:, idx] - v_pred, axis=0) <= 1e-5 * scale)
    # touching partners of the sample from the production contact kernel's
    # pair output, on the sorted input state
    T.say(f"[full size] {name}: pair sets of the sample")
    cur, nxt = sim.cur, sim.nxt
    X0 = T.dev(x.reshape(-1))
    gic.gic_sort_cells(sim.ctx, X0.view(3, n), s["key"], s["order"], s["cell_begin"], s["cell_end"])
    ID0 = torch.arange(n, dtype=torch.int32, device="cuda")
    gic.gic_reorder(sim.ctx, s["order"], X0.view(3, n), T.dev(v.reshape(-1)), T.dev(r), ID0, nxt["x"], nxt["v"],
                    nxt["r"], nxt["id"])
    del X0
    cap = 16
    PR = torch.empty(cap * n, dtype=torch.int32, device="cuda")
    gic.gic_contact_forces(sim.ctx, nxt["x"], nxt["v"], nxt["r"], s["cell_begin"], s["cell_end"], s["f_contact"],
                           pair_ids=PR)
    torch.cuda.synchronize()
    ids = nxt["id"].cpu().numpy()
    sp = np.empty(n, np.int64)
    sp[ids] = np.arange(n)
    P = PR.view(cap, n)[:, torch.as_tensor(sp[idx], device="cuda")].cpu().numpy()
    del PR
    got = [set(ids[P[:, k][P[:, k] >= 0]].tolist()) for k in range(idx.size)]
    ref = orc.pairs_sample(cfg, x, r, idx)
    assert got == ref and sum(map(len, ref)) > 0
    if name == "c3":
        # P2G of the oracle's advanced state (every granule) through the HIP path
        T.say(f"[full size] {name}: oracle step of every granule")
        st = orc.step(cfg, x, v, r, u, a0)
        a1g, m1g = T.p2g_of(cfg, st["x"], st["v"], r, "fp32", r_max=float(r.max()))
        assert np.array_equal(a1g, st["alpha"]) and np.array_equal(m1g, st["mom"])
    T.say(f"[full size] {name}: ok, contacts in sample {int((fa > 0).sum())}")


def test_full_size_wet_bed(T, orc):
    """The c3 bed wet (seeded moisture ratios U(0, 1), held water U(0, 0.3)
    per granule volume, so wet masses in the damping): the input state
    sorted and reordered as a step begins, then the contact plus
    liquid-bridge call on it, launched as the benchmark's wet-bed leg does;
    sampled forces against the oracle's contact plus capillary forces of the
    same state (computed one by one), to the 1e-5 FP32-form bar of the
    summed term magnitudes."""
    import torch
    from paper_2504_00745_amd import gic
    T.say("[full size] c3 wet bed: generating")
    d = wl.make("c3")
    cfg = dict(d["params"], sigma=0.072, vbridge=1e-4, sr_peak=0.3)
    x, v, r, u = d["x"], d["v"], d["r"], d["u"]
    n = x.shape[1]
    rng = np.random.Generator(np.random.PCG64(17))
    sr = rng.uniform(0.0, 1.0, n).astype(np.float32).astype(np.float64)  # the FP32 form's values
    held = rng.uniform(0.0, 0.3, n)  # water held per granule volume: wet masses (Eq. 19)
    cfg["rho_f"] = 1000.0
    sim = gic.Simulator(cfg, x, v, r, u, "fp32", r_max=float(r.max()))
    ctx, s = sim.ctx, sim.scratch
    cur, nxt = sim.cur, sim.nxt
    # sort and reorder the input state as a step does, then the wet contact call
    gic.gic_sort_cells(ctx, cur["x"], s["key"], s["order"], s["cell_begin"], s["cell_end"])
    gic.gic_reorder(ctx, s["order"], cur["x"], cur["v"], cur["r"], cur["id"], nxt["x"], nxt["v"], nxt["r"],
                    nxt["id"])
    ids = nxt["id"].long()
    SR = torch.as_tensor(sr, dtype=torch.float32, device="cuda")[ids].contiguous()
    H = torch.as_tensor(held, dtype=torch.float64, device="cuda")[ids].contiguous()
    F = torch.empty(3 * n, dtype=torch.float32, device="cuda")
    T.say("[full size] c3 wet bed: GPU contact + bridges")
    gic.gic_contact_capillary_forces(ctx, nxt["x"], nxt["v"], nxt["r"], SR, s["cell_begin"], s["cell_end"], F,
                                     held=H)
    torch.cuda.synchronize()
    assert ctx.error() == (0, -1)
    idv = ids.cpu().numpy()
    pos = np.empty(n, np.int64)
    pos[idv] = np.arange(n)
    idx = rng.choice(n, 3000, replace=False)
    T.say("[full size] c3 wet bed: oracle samples")
    Fs, fa = orc.contact_forces_sample_wet(cfg, x, v, r, orc.wet_mass(cfg, r, held), idx)
    Fb, fb = orc.capillary_forces_sample(cfg, x, r, sr, idx)
    Fg = F.view(3, n).double().cpu().numpy()[:, pos[idx]]
    err = np.linalg.norm(Fg - (Fs + Fb), axis=0)
    S = fa + fb
    assert np.all(err <= 1e-5 * S + 1e-300), np.max(err / (S + 1e-300))
    T.say(f"[full size] c3 wet bed: ok, bridged granules in sample {int((fb > 0).sum())}")
