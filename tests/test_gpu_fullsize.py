"""Parity at full workload sizes, in the launch configuration bench.py times
(one gic_step of the Simulator, FP32 form):

  c3: 4,194,304 granules, 256x128x128 grid (the benchmark workload)
  c5: 16,777,216 granules, 512x256x256 grid (the largest)

Checked: cell keys, sort order and cell ranges bit-exact against the oracle
over all granules; the int64 P2G grids of the GPU's advanced state bit-exact
against the oracle over the whole grid; contact forces and advanced
velocities of a random sample of granules against the oracle (computed one
by one), to the 1e-5 FP32-form bar of the pair-force sums.
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
    # P2G of the advanced state, whole grid
    x1, v1 = sim.state_in_input_order()
    T.say(f"[full size] {name}: oracle P2G")
    a1, m1 = orc.p2g_fixed(cfg, x1, v1, r)
    assert np.array_equal(sim.alpha.cpu().numpy(), a1)
    assert np.array_equal(sim.mom.cpu().numpy().reshape(3, -1), m1)
    del a1, m1
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
    Fd = s["f_drag"].view(3, n).double().cpu().numpy()[:, pos[idx]]
    g = np.array(cfg["g"])[:, None]
    v_pred = v[:, idx] + cfg["dt"] * ((Fs + Fd) / m + g)
    scale = np.linalg.norm(v_pred, axis=0) + cfg["dt"] * (fa + np.linalg.norm(Fd, axis=0) + m * 9.81) / m
    assert np.all(np.linalg.norm(v1[:, idx] - v_pred, axis=0) <= 1e-5 * scale)
    T.say(f"[full size] {name}: ok, contacts in sample {int((fa > 0).sum())}")
