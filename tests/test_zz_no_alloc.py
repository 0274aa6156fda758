"""gic_sum_noalloc, the allocation-free variant of gic_sum: its partial sums
live in a fixed array the library holds per device.  Two calls in a row,
the second on a smaller input (the array keeps the first call's partials),
plain sums and dot products, with and without accumulation: each equals
gic_sum of the same input bit for bit (same kernels, same order)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_sum_noalloc_equals_sum():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_00745_amd import gic
    from paper_2504_00745_amd import workloads as wl
    d = wl.make("c1")
    ctx = gic.Context(d["params"], 8, "fp64")
    rng = np.random.Generator(np.random.PCG64(11))
    for n in (3_000_017, 40_000, 1):  # each call after a larger one
        print(f"[no-alloc] n={n}", flush=True)
        a = torch.as_tensor(rng.standard_normal(n) * 1e3, device="cuda")
        b = torch.as_tensor(rng.uniform(-1.0, 1.0, n), device="cuda")
        for bb in (None, b):
            ref = torch.full((1,), 0.25, dtype=torch.float64, device="cuda")
            got = torch.full((1,), 0.25, dtype=torch.float64, device="cuda")
            gic.gic_sum(ctx, a, ref, b=bb, accumulate=True)
            gic.gic_sum_noalloc(a, got, b=bb, accumulate=True)
            assert torch.equal(got, ref)
            gic.gic_sum(ctx, a, ref, b=bb)
            gic.gic_sum_noalloc(a, got, b=bb)
            torch.cuda.synchronize()
            assert torch.equal(got, ref)
            exact = float(np.sum((a * bb if bb is not None else a).cpu().numpy().astype(np.longdouble)))
            assert abs(float(got) - exact) <= 1e-12 * float((a.abs() * (bb.abs() if bb is not None else 1)).sum())
    # the empty sum, and the argument checks (no kernel runs)
    z = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    gic.gic_sum_noalloc(torch.empty(0, dtype=torch.float64, device="cuda"), z)
    torch.cuda.synchronize()
    assert float(z) == 0.0
    L = gic.lib()
    assert L.gic_sum_noalloc(-1, None, None, gic._ptr(z), 0, None) != 0
    assert L.gic_sum_noalloc((1 << 30) + 1, gic._ptr(z), None, gic._ptr(z), 0, None) != 0
    assert L.gic_sum_noalloc(4, gic._ptr(z), None, None, 0, None) != 0
