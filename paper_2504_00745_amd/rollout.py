"""Differentiable rollout of the granule step on the GPU (double precision).

Forward, per step (unquantised transfers, Sec. 5.1 Eq. 7a, Sec. 5.2):
    A = P2G_alpha(x);  (u_at, alpha_f) = G2P(x; u, A);
    F_d = C_d 6 pi eta r alpha_f (u_at - v);  F_c = contact(x, v; mu)  (Eq. 1);
    v' = v + dt ((F_c + F_d)/m + g);  x' = x + dt v'       (Sec. 4);
loss L = sum_k |P_k|^2 with P = P2G_momentum(x_T, v_T) in kg m/s.

GICRollout is a torch.autograd.Function whose backward runs the adjoint
kernels of the C ABI (gic_*_vjp): states are checkpointed every `ckpt`
steps in the forward, each segment is recomputed in the backward and walked
in reverse.  The granule state is kept in input order; each step sorts, works
on a sorted copy and scatters the result back, so adjoints are gathered and
scattered with the same permutations.  PyTorch provides device memory and
the stream only: the loss cotangent is scaled on the device (gic_scale) and
the parameters mu and c_drag, kernel arguments, are read from host tensors
(or numbers), so neither pass reads the device back.

With graph=True each pass is recorded once as a HIP graph (through
torch.cuda.CUDAGraph: every launch of the pass, a few hundred, becomes one
replay) and replayed with its inputs copied into the recorded buffers; it is
recorded again when mu or c_drag change, since they are captured as kernel
arguments.  The kernels are deterministic, so a replay gives the bits of the
direct run.
"""
import torch

from . import gic


class Rollout:
    """Buffers and parameters of a differentiable rollout."""

    def __init__(self, cfg, r, u, steps, ckpt=5, r_max=None, graph=False):
        self.graph = bool(graph)
        self._fwd = None  # (params, graph, static inputs, static outputs) of the recorded forward
        self._bwd = None
        self.n = int(r.shape[-1])
        self.steps = int(steps)
        self.ckpt = int(ckpt)
        self.ctx = gic.Context(cfg, self.n, "fp64", r_max)
        dev = torch.device("cuda")
        f64 = torch.float64
        n, G, K = self.n, self.ctx.G, self.ctx.K
        self.r = torch.as_tensor(r, dtype=f64).to(dev).contiguous()
        self.u = torch.as_tensor(u, dtype=f64).to(dev).contiguous().view(-1)
        e = lambda *s, dt=f64: torch.empty(*s, dtype=dt, device=dev)
        self.key, self.order = e(n, dt=torch.int32), e(n, dt=torch.int32)
        self.cb, self.ce = e(K, dt=torch.int32), e(K, dt=torch.int32)
        self.xs, self.vs, self.rs = e(3 * n), e(3 * n), e(n)
        self.A, self.gA = e(G), e(G)
        self.P = e(3 * G)
        self.uat, self.af, self.Fd, self.Fc = e(3 * n), e(n), e(3 * n), e(3 * n)
        self.gxs, self.gvs, self.gF = e(3 * n), e(3 * n), e(3 * n)
        self.guat, self.gaf, self.gmu_i, self.gcd_i = e(3 * n), e(n), e(n), e(n)
        self.scal = torch.zeros(4, dtype=f64, device=dev)  # L, dL/dmu, dL/dC_d, spare
        self.params = (float(cfg["mu"]), float(cfg["c_drag"]))

    def set_params(self, mu, c_drag):
        self.params = (float(mu), float(c_drag))
        self.ctx.set_params(mu=self.params[0], c_drag=self.params[1])

    # ---- forward pieces --------------------------------------------------
    def _sorted(self, x, v):
        """Sort by cell, gather x, v, r into sorted order (one kernel)."""
        c = self.ctx
        gic.gic_sort_cells(c, x.view(3, -1), self.key, self.order, self.cb, self.ce)
        gic.gic_reorder(c, self.order, x.view(3, -1), v, self.r, None, self.xs, self.vs, self.rs, None)

    def _forces(self):
        c = self.ctx
        xs = self.xs.view(3, -1)
        gic.gic_p2g_real(c, xs, self.vs, self.rs, self.cb, self.ce, self.A, None)
        gic.gic_g2p(c, xs, self.u, None, self.A, self.uat, self.af)
        gic.gic_drag(c, self.rs, self.vs, self.uat, self.af, self.Fd)

    def step(self, x, v, x_out, v_out):
        """One step from (x, v) (input order) into (x_out, v_out)."""
        c = self.ctx
        self._sorted(x, v)
        self._forces()
        gic.gic_contact_forces(c, self.xs.view(3, -1), self.vs, self.rs, self.cb, self.ce, self.Fc)
        gic.gic_integrate(c, self.rs, self.Fc, self.Fd, self.xs, self.vs)
        gic.gic_permute(c, self.order, self.xs, x_out, 3, True)
        gic.gic_permute(c, self.order, self.vs, v_out, 3, True)

    def loss(self, x, v):
        """L = sum |P|^2 of the momentum grid of (x, v), into self.scal[0]."""
        c = self.ctx
        self._sorted(x, v)
        gic.gic_p2g_real(c, self.xs.view(3, -1), self.vs, self.rs, self.cb, self.ce, None, self.P)
        gic.gic_sum(c, self.P, self.scal[0:1], b=self.P)

    def forward(self, x0, v0):
        """Runs the rollout; returns the loss tensor (1,), the checkpoints
        and the final state (tensors of their own)."""
        if not self.graph:
            return self._forward(x0, v0)
        x0, v0 = x0.detach().reshape(-1), v0.detach().reshape(-1)
        if self._fwd is None or self._fwd[0] != self.params:
            sx, sv = x0.clone(), v0.clone()
            out = self._record(lambda: self._forward(sx, sv))
            self._fwd = (self.params, out[0], (sx, sv), out[1])
        _, g, (sx, sv), (L, ckpts, final) = self._fwd
        sx.copy_(x0)
        sv.copy_(v0)
        g.replay()
        return L.clone(), [(a.clone(), b.clone()) for a, b in ckpts], (final[0].clone(), final[1].clone())

    @staticmethod
    def _record(fn):
        """fn run once directly (warm-up), then recorded as a graph; returns
        (graph, fn's outputs in the graph's memory)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fn()
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            out = fn()
        return g, out

    def _forward(self, x0, v0):
        x, v = x0.contiguous().clone().view(-1), v0.contiguous().clone().view(-1)
        x2, v2 = torch.empty_like(x), torch.empty_like(v)
        ckpts = []
        for s in range(self.steps):
            if s % self.ckpt == 0:
                ckpts.append((x.clone(), v.clone()))
            self.step(x, v, x2, v2)
            x, x2, v, v2 = x2, x, v2, v
        self.loss(x, v)
        return self.scal[0:1].clone(), ckpts, (x, v)

    # ---- reverse pass ----------------------------------------------------
    def backward(self, ckpts, final, gL):
        """Gradients (dL/dv0 (3,n), dL/dmu, dL/dC_d) for cotangent gL of L."""
        if not self.graph:
            return self._backward(ckpts, final, gL)
        gL = gL.detach().reshape(1).to(torch.float64)
        if self._bwd is None or self._bwd[0] != self.params or len(self._bwd[2][0]) != len(ckpts):
            sc = [(a.clone(), b.clone()) for a, b in ckpts]
            sf = (final[0].clone(), final[1].clone())
            sg = gL.clone()
            out = self._record(lambda: self._backward(sc, sf, sg))
            self._bwd = (self.params, out[0], (sc, sf, sg), out[1])
        _, g, (sc, sf, sg), (gv, gmu, gcd) = self._bwd
        for (a, b), (c, d) in zip(sc, ckpts):
            a.copy_(c)
            b.copy_(d)
        sf[0].copy_(final[0])
        sf[1].copy_(final[1])
        sg.copy_(gL)
        g.replay()
        return gv.clone(), gmu.clone(), gcd.clone()

    def _backward(self, ckpts, final, gL):
        c = self.ctx
        n = self.n
        x, v = final
        gx = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
        gv = torch.zeros_like(gx)
        self.scal[1:3].zero_()
        # L = sum P^2  ->  dL/dP = 2 gL P, gL a device scalar
        self.loss(x, v)
        gP = torch.empty_like(self.P)
        gic.gic_scale(c, self.P, gL.reshape(1).to(torch.float64), 2.0, gP)
        self.gxs.zero_()
        self.gvs.zero_()
        gic.gic_p2g_vjp(c, self.xs.view(3, -1), self.vs, self.rs, None, gP, self.gxs, self.gvs)
        gic.gic_permute(c, self.order, self.gxs, gx, 3, True)
        gic.gic_permute(c, self.order, self.gvs, gv, 3, True)
        nseg = len(ckpts)
        for seg in reversed(range(nseg)):
            s0 = seg * self.ckpt
            s1 = min(s0 + self.ckpt, self.steps)
            xs_list = [ckpts[seg]]
            xa, va = ckpts[seg][0].clone(), ckpts[seg][1].clone()
            for s in range(s0, s1 - 1):
                xb, vb = torch.empty_like(xa), torch.empty_like(va)
                self.step(xa, va, xb, vb)
                xs_list.append((xb, vb))
                xa, va = xb, vb
            for s in reversed(range(s0, s1)):
                xn, vn = xs_list[s - s0]
                self._sorted(xn, vn)
                self._forces()
                gic.gic_permute(c, self.order, gx, self.gxs, 3, False)
                gic.gic_permute(c, self.order, gv, self.gvs, 3, False)
                xs = self.xs.view(3, -1)
                gic.gic_integrate_vjp(c, self.rs, self.gxs, self.gvs, self.gF)
                gic.gic_contact_forces_vjp(c, xs, self.vs, self.rs, self.cb, self.ce, self.gF, self.gxs, self.gvs,
                                           self.gmu_i)
                gic.gic_sum(c, self.gmu_i, self.scal[1:2], accumulate=True)
                gic.gic_drag_vjp(c, self.rs, self.vs, self.uat, self.af, self.gF, self.gvs, self.guat, self.gaf,
                                 self.gcd_i)
                gic.gic_sum(c, self.gcd_i, self.scal[2:3], accumulate=True)
                gic.gic_g2p_vjp(c, xs, self.u, self.A, self.guat, self.gaf, self.cb, self.ce, self.gxs, self.gA)
                gic.gic_p2g_vjp(c, xs, self.vs, self.rs, self.gA, None, self.gxs, self.gvs)
                gic.gic_permute(c, self.order, self.gxs, gx, 3, True)
                gic.gic_permute(c, self.order, self.gvs, gv, 3, True)
        return gv.view(3, n), self.scal[1:2].clone(), self.scal[2:3].clone()


class GICRollout(torch.autograd.Function):
    """L = rollout loss; differentiable in v0, mu and c_drag."""

    @staticmethod
    def forward(ctx, x0, v0, mu, c_drag, sim):
        # mu and c_drag are kernel arguments: host values (CPU tensors or
        # numbers), read without a device synchronisation
        sim.set_params(float(mu.detach().cpu()) if mu.is_cuda else float(mu),
                       float(c_drag.detach().cpu()) if c_drag.is_cuda else float(c_drag))
        L, ckpts, final = sim.forward(x0, v0)
        ctx.sim = sim
        ctx.ckpts = ckpts
        ctx.final = final
        return L.view(())

    @staticmethod
    def backward(ctx, gL):
        gv0, gmu, gcd = ctx.sim.backward(ctx.ckpts, ctx.final, gL)
        return None, gv0, gmu.view(()), gcd.view(()), None
