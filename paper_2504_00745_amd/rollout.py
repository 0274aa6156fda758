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
scattered with the same permutations.  Positions and velocities (and their
adjoints) share one buffer, x then v (6n doubles), so each gather or scatter
of both is one gic_permute of six components.  PyTorch provides device memory and
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
        self.xvs, self.rs = e(6 * n), e(n)  # sorted x then v
        self.xs, self.vs = self.xvs[:3 * n], self.xvs[3 * n:]
        self.A, self.gA = e(G), e(G)
        self.P = e(3 * G)
        self.uat, self.af, self.Fd, self.Fc = e(3 * n), e(n), e(3 * n), e(3 * n)
        self.gxvs, self.gF = e(6 * n), e(3 * n)  # sorted adjoints of x then v
        self.gxs, self.gvs = self.gxvs[:3 * n], self.gxvs[3 * n:]
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
        gic.gic_brick_list(c, self.cb, self.ce)  # one brick schedule for the step's brick kernels
        gic.gic_reorder(c, self.order, x.view(3, -1), v, self.r, None, self.xs, self.vs, self.rs, None)

    def _forces(self):
        c = self.ctx
        xs = self.xs.view(3, -1)
        gic.gic_p2g_real(c, xs, self.vs, self.rs, self.cb, self.ce, self.A, None)
        gic.gic_g2p(c, xs, self.u, None, self.A, self.uat, self.af)
        gic.gic_drag(c, self.rs, self.vs, self.uat, self.af, self.Fd)

    def _split(self, xv):
        return xv[:3 * self.n], xv[3 * self.n:]

    def step(self, xv, xv_out):
        """One step from the state xv = (x, v) (input order) into xv_out."""
        c = self.ctx
        self._sorted(*self._split(xv))
        self._forces()
        gic.gic_contact_forces(c, self.xs.view(3, -1), self.vs, self.rs, self.cb, self.ce, self.Fc)
        gic.gic_integrate(c, self.rs, self.Fc, self.Fd, self.xs, self.vs)
        gic.gic_permute(c, self.order, self.xvs, xv_out, 6, True)

    def loss(self, xv):
        """L = sum |P|^2 of the momentum grid of the state xv, into self.scal[0]."""
        c = self.ctx
        self._sorted(*self._split(xv))
        gic.gic_p2g_real(c, self.xs.view(3, -1), self.vs, self.rs, self.cb, self.ce, None, self.P)
        gic.gic_sum(c, self.P, self.scal[0:1], b=self.P)

    def forward(self, x0, v0):
        """Runs the rollout; returns the loss tensor (1,), the checkpoints
        and the final state (states (x, v) as one tensor of 6n, of their
        own)."""
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
        return L.clone(), [a.clone() for a in ckpts], final.clone()

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
        xv = torch.cat([x0.reshape(-1), v0.reshape(-1)])
        xv2 = torch.empty_like(xv)
        ckpts = []
        for s in range(self.steps):
            if s % self.ckpt == 0:
                ckpts.append(xv.clone())
            self.step(xv, xv2)
            xv, xv2 = xv2, xv
        self.loss(xv)
        return self.scal[0:1].clone(), ckpts, xv

    # ---- reverse pass ----------------------------------------------------
    def backward(self, ckpts, final, gL):
        """Gradients (dL/dv0 (3,n), dL/dmu, dL/dC_d) for cotangent gL of L."""
        if not self.graph:
            return self._backward(ckpts, final, gL)
        gL = gL.detach().reshape(1).to(torch.float64)
        if self._bwd is None or self._bwd[0] != self.params or len(self._bwd[2][0]) != len(ckpts):
            sc = [a.clone() for a in ckpts]
            sf = final.clone()
            sg = gL.clone()
            out = self._record(lambda: self._backward(sc, sf, sg))
            self._bwd = (self.params, out[0], (sc, sf, sg), out[1])
        _, g, (sc, sf, sg), (gv, gmu, gcd) = self._bwd
        for a, c in zip(sc, ckpts):
            a.copy_(c)
        sf.copy_(final)
        sg.copy_(gL)
        g.replay()
        return gv.clone(), gmu.clone(), gcd.clone()

    def _backward(self, ckpts, final, gL):
        c = self.ctx
        n = self.n
        gxv = torch.zeros(6 * n, dtype=torch.float64, device="cuda")  # adjoint of (x, v), input order
        self.scal[1:3].zero_()
        # L = sum P^2  ->  dL/dP = 2 gL P, gL a device scalar
        self.loss(final)
        gP = torch.empty_like(self.P)
        gic.gic_scale(c, self.P, gL.reshape(1).to(torch.float64), 2.0, gP)
        self.gxvs.zero_()
        gic.gic_p2g_vjp(c, self.xs.view(3, -1), self.vs, self.rs, None, gP, self.gxs, self.gvs)
        gic.gic_permute(c, self.order, self.gxvs, gxv, 6, True)
        nseg = len(ckpts)
        for seg in reversed(range(nseg)):
            s0 = seg * self.ckpt
            s1 = min(s0 + self.ckpt, self.steps)
            xs_list = [ckpts[seg]]
            xa = ckpts[seg].clone()
            for s in range(s0, s1 - 1):
                xb = torch.empty_like(xa)
                self.step(xa, xb)
                xs_list.append(xb)
                xa = xb
            for s in reversed(range(s0, s1)):
                self._sorted(*self._split(xs_list[s - s0]))
                self._forces()
                gic.gic_permute(c, self.order, gxv, self.gxvs, 6, False)
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
                gic.gic_permute(c, self.order, self.gxvs, gxv, 6, True)
        return gxv[3 * n:].view(3, n), self.scal[1:2].clone(), self.scal[2:3].clone()


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
