"""Helpers of the GPU parity tests: run the HIP stages through the C ABI on
seeded inputs and bring the results back in the oracle's (input) order."""
import sys

import numpy as np
import torch

from paper_2504_00745_amd import gic


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dtype).contiguous()


def run_stages(cfg, x, v, r, u, precision, alpha_in=None, r_max=None):
    """One sub-step through the separate entry points.  Returns numpy arrays
    in input order: key, order, cell ranges, and per stage outputs."""
    n = x.shape[1]
    ctx = gic.Context(cfg, max(n, 1), precision, r_max)
    real = ctx.real
    X, V, R = dev(x.reshape(-1)), dev(v.reshape(-1)), dev(r)
    ID = torch.arange(n, dtype=torch.int32, device="cuda")
    key = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    order = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    cb = torch.empty(ctx.K, dtype=torch.int32, device="cuda")
    ce = torch.empty(ctx.K, dtype=torch.int32, device="cuda")
    gic.gic_sort_cells(ctx, X.view(3, n), key, order, cb, ce)
    Xs, Vs, Rs, IDs = torch.empty_like(X), torch.empty_like(V), torch.empty_like(R), torch.empty_like(ID)
    gic.gic_reorder(ctx, order, X.view(3, n), V, R, ID, Xs, Vs, Rs, IDs)
    out = dict(ctx=ctx, key=key[:n].cpu().numpy().view(np.uint32), order=order[:n].cpu().numpy(),
               cell_begin=cb.cpu().numpy(), cell_end=ce.cpu().numpy(), ids=IDs.cpu().numpy())
    U = dev(u.reshape(-1), real)
    if alpha_in is None:
        A0 = torch.zeros(ctx.G, dtype=torch.int64, device="cuda")
        gic.gic_p2g(ctx, Xs.view(3, n), Vs, Rs, cb, ce, A0, None)
    else:
        A0 = dev(alpha_in, torch.int64)
    out["alpha0"] = A0.cpu().numpy()
    uat = torch.empty(3 * n, dtype=real, device="cuda")
    af = torch.empty(n, dtype=real, device="cuda")
    gic.gic_g2p(ctx, Xs.view(3, n), U, A0, None, uat, af)
    Fd = torch.empty(3 * n, dtype=real, device="cuda")
    gic.gic_drag(ctx, Rs, Vs, uat, af, Fd)
    Fc = torch.empty(3 * n, dtype=real, device="cuda")
    nct = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    pairs = torch.empty(PAIR_CAP * max(n, 1), dtype=torch.int32, device="cuda")
    gic.gic_contact_forces(ctx, Xs.view(3, n), Vs, Rs, cb, ce, Fc, nct, pair_ids=pairs[:PAIR_CAP * n])
    X1, V1 = Xs.clone(), Vs.clone()
    gic.gic_integrate(ctx, Rs, Fc, Fd, X1, V1)
    A1 = torch.empty(ctx.G, dtype=torch.int64, device="cuda")
    M1 = torch.empty(3 * ctx.G, dtype=torch.int64, device="cuda")
    gic.gic_p2g(ctx, X1.view(3, n), V1, Rs, cb, ce, A1, M1)
    torch.cuda.synchronize()
    ids = out["ids"]

    def unsort(t, comps):
        a = t.double().cpu().numpy().reshape(comps, n) if comps > 1 else t.double().cpu().numpy()[:n]
        o = np.empty_like(a)
        if comps > 1:
            o[:, ids] = a
        else:
            o[ids] = a
        return o

    out["pairs"] = pair_set(pairs[:PAIR_CAP * n].cpu().numpy().reshape(PAIR_CAP, n), ids)
    out.update(u_at=unsort(uat, 3), alpha_f=unsort(af, 1), Fd=unsort(Fd, 3), Fc=unsort(Fc, 3),
               ncont=unsort(nct[:n], 1).astype(np.int64), x1=unsort(X1, 3), v1=unsort(V1, 3),
               alpha1=A1.cpu().numpy(), mom1=M1.cpu().numpy().reshape(3, -1), err=ctx.error())
    return out


PAIR_CAP = 32  # touching partners kept per granule by the pair output of gic_contact_forces


def pair_set(P, ids):
    """Set of touching pairs (i, j), i < j, in input indices, from the pair
    output of gic_contact_forces (P: cap x n sorted positions, -1 after the
    last; ids[q] = input index at sorted position q).  Every pair must be
    listed from both of its granules."""
    cap, n = P.shape
    mask = P >= 0
    q = np.nonzero(mask)[1]
    j = P[mask]
    a, b = ids[q], ids[j]
    directed = set(zip(a.tolist(), b.tolist()))
    assert len(directed) == q.size, "a partner listed twice"
    assert all((y, x) in directed for x, y in directed), "a pair listed from one side only"
    return set((min(x, y), max(x, y)) for x, y in directed)


def p2g_of(cfg, x, v, r, precision, r_max=None):
    """int64 P2G grids (alpha (G,), momentum (3, G)) of a host state through
    the HIP path (sort, reorder, gic_p2g)."""
    n = x.shape[1]
    ctx = gic.Context(cfg, max(n, 1), precision, r_max)
    X, V, R = dev(x.reshape(-1)), dev(v.reshape(-1)), dev(r)
    ID = torch.arange(n, dtype=torch.int32, device="cuda")
    key = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    order = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    cb = torch.empty(ctx.K, dtype=torch.int32, device="cuda")
    ce = torch.empty(ctx.K, dtype=torch.int32, device="cuda")
    gic.gic_sort_cells(ctx, X.view(3, n), key, order, cb, ce)
    Xs, Vs, Rs, IDs = torch.empty_like(X), torch.empty_like(V), torch.empty_like(R), torch.empty_like(ID)
    gic.gic_reorder(ctx, order, X.view(3, n), V, R, ID, Xs, Vs, Rs, IDs)
    A = torch.zeros(ctx.G, dtype=torch.int64, device="cuda")
    M = torch.zeros(3 * ctx.G, dtype=torch.int64, device="cuda")
    gic.gic_p2g(ctx, Xs.view(3, n), Vs, Rs, cb, ce, A, M)
    torch.cuda.synchronize()
    return A.cpu().numpy(), M.cpu().numpy().reshape(3, -1)
