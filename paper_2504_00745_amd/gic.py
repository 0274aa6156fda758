"""Thin Python binding of the gfx950 C ABI (include/gic.h).

Argument marshalling only: torch tensors on the GPU provide device memory
and torch's current stream is passed to every call; every step of the path
runs in the HIP kernels of libgic.so.  Functions keep the C names.  A missing
library raises immediately: there is no fallback.
"""
import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgic.so")
_LIB = None

GIC_FP64 = 0
GIC_FP32 = 1
STATUS = {0: "GIC_OK", 1: "GIC_E_ARG", 2: "GIC_E_HIP", 3: "GIC_E_ALLOC", 4: "GIC_E_DOMAIN", 5: "GIC_E_NONFINITE",
          6: "GIC_E_RANGE"}


class GicError(RuntimeError):
    def __init__(self, status, where):
        super().__init__(f"{where}: {STATUS.get(status, status)}")
        self.status = status


class gic_params(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3), ("pad0", C.c_int32), ("dx", C.c_double),
        ("nc", C.c_int32 * 3), ("pad1", C.c_int32), ("cell", C.c_double),
        ("kn", C.c_double), ("restitution", C.c_double), ("kt_ratio", C.c_double), ("mu", C.c_double),
        ("rho_s", C.c_double), ("eta_f", C.c_double), ("c_drag", C.c_double), ("alpha_max", C.c_double),
        ("g", C.c_double * 3), ("dt", C.c_double), ("r_max", C.c_double),
        ("walls", C.c_uint32), ("precision", C.c_int32),
        ("rho_f", C.c_double), ("c_quad", C.c_double), ("f_unit", C.c_double),
        ("drag_model", C.c_int32), ("vmass", C.c_int32),
        ("sigma", C.c_double), ("vbridge", C.c_double), ("sr_peak", C.c_double),
        ("absorb_max", C.c_double),
    ]


_V = C.c_void_p
_I64 = C.c_int64
_I32 = C.c_int32
_PP = C.POINTER(gic_params)


def lib():
    """The loaded libgic.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2504_00745_amd.build`")
        L = C.CDLL(LIB_PATH)
        sig = {
            "gic_key_space": (_I64, [_PP]),
            "gic_create": (C.c_int, [_PP, _I64, C.POINTER(_V)]),
            "gic_set_params": (C.c_int, [_V, _PP]),
            "gic_destroy": (C.c_int, [_V]),
            "gic_get_error": (C.c_int, [_V, _V, C.POINTER(_I32), C.POINTER(_I64), _I32]),
            "gic_neighbour_builds": (C.c_int, [_V, _V, C.POINTER(_I64)]),
            "gic_stage_timing": (C.c_int, [_V, _I32]),
            "gic_stage_times": (C.c_int, [_V, _V, C.POINTER(C.c_double), C.POINTER(_I32)]),
            "gic_sort_cells": (C.c_int, [_V, _I64, _V, _V, _V, _V, _V, _V]),
            "gic_brick_list": (C.c_int, [_V, _V, _V, _V]),
            "gic_reorder": (C.c_int, [_V, _I64, _V, _V, _V, _V, _V, _V, _V, _V, _V, _V]),
            "gic_contact_forces": (C.c_int, [_V, _I64, _V, _V, _V, _V, _V, _V, _V, _V, _I32, _V]),
            "gic_contact_capillary_forces": (C.c_int, [_V, _I64, _V, _V, _V, _V, _V, _V, _V, _V, _V, _V]),
            "gic_integrate_p2g_wet": (C.c_int, [_V, _I64, _V, _V, _V, _V, _V, _V, _V, _V, _V, _V, _I32, _V]),
            "gic_moisture_ratio": (C.c_int, [_V, _I64, _V, _V, _V, _V]),
            "gic_idp_workspace_bytes": (_I64, [_V]),
            "gic_idp_setup": (C.c_int, [_V] * 7),
            "gic_idp_apply": (C.c_int, [_V] * 6),
            "gic_idp_solve": (C.c_int, [_V] * 6 + [_I32, C.c_double, _I32, _I32, _V, _V, _V]),
            "gic_idp_displacement": (C.c_int, [_V] * 7),
            "gic_density_projection": (C.c_int, [_V] * 9 + [_I32, C.c_double, _I32, _I32, _V, _V, _V]),
            "gic_g2p": (C.c_int, [_V, _I64, _V, _V, _V, _V, _V, _V, _V]),
            "gic_drag": (C.c_int, [_V, _I64, _V, _V, _V, _V, _V, _V]),
            "gic_integrate": (C.c_int, [_V, _I64, _V, _V, _V, _V, _V, _V]),
            "gic_p2g": (C.c_int, [_V, _I64, _V, _V, _V, _V, _V, _V, _V, _I32, _V]),
            "gic_p2g_real": (C.c_int, [_V, _I64, _V, _V, _V, _V, _V, _V, _V, _I32, _V]),
            "gic_gather_g2p_drag": (C.c_int, [_V, _I64] + [_V] * 17),
            "gic_integrate_p2g": (C.c_int, [_V, _I64] + [_V] * 9 + [_I32, _V]),
            "gic_step": (C.c_int, [_V, _I64] + [_V] * 20),
            "gic_gather_g2p_fluid": (C.c_int, [_V, _I64] + [_V] * 19),
            "gic_exchange_p2g": (C.c_int, [_V, _I64] + [_V] * 6 + [C.c_double, _V, _V, _V]),
            "gic_sand_step": (C.c_int, [_V, _I64, C.c_double] + [_V] * 23),
            "gic_contact_forces_vjp": (C.c_int, [_V, _I64] + [_V] * 10),
            "gic_drag_vjp": (C.c_int, [_V, _I64] + [_V] * 10),
            "gic_integrate_vjp": (C.c_int, [_V, _I64] + [_V] * 5),
            "gic_g2p_vjp": (C.c_int, [_V, _I64] + [_V] * 10),
            "gic_p2g_vjp": (C.c_int, [_V, _I64] + [_V] * 8),
            "gic_sum": (C.c_int, [_V, _I64, _V, _V, _V, _I32, _V]),
            "gic_sum_noalloc": (C.c_int, [_I64, _V, _V, _V, _I32, _V]),
            "gic_permute": (C.c_int, [_V, _I64, _I32, _V, _V, _V, _I32, _V]),
            "gic_scale": (C.c_int, [_V, _I64, _V, _V, C.c_double, _V, _V]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def make_params(cfg: dict, precision: str = "fp32", r_max: float = None) -> gic_params:
    """C parameter block from a workload parameter dict (workloads.spec)."""
    p = gic_params()
    p.n = (C.c_int32 * 3)(*cfg["n"])
    p.dx = float(cfg["dx"])
    p.nc = (C.c_int32 * 3)(*cfg["nc"])
    p.cell = float(cfg["cell"])
    for k in ("kn", "restitution", "kt_ratio", "mu", "rho_s", "eta_f", "c_drag", "alpha_max", "dt"):
        setattr(p, k, float(cfg[k]))
    p.g = (C.c_double * 3)(*cfg["g"])
    p.r_max = float(cfg["cell"] / 2.0 if r_max is None else r_max)
    p.walls = int(cfg["walls"])
    p.precision = GIC_FP32 if precision == "fp32" else GIC_FP64
    # remaining interphase forces: off unless the workload sets them
    p.rho_f = float(cfg.get("rho_f", 0.0))
    p.c_quad = float(cfg.get("c_quad", 0.0))
    p.f_unit = float(cfg.get("f_unit", 1.0))
    p.drag_model = int(cfg.get("drag_model", 0))
    p.vmass = int(cfg.get("vmass", 0))
    p.sigma = float(cfg.get("sigma", 0.0))
    p.vbridge = float(cfg.get("vbridge", 1e-4))
    p.sr_peak = float(cfg.get("sr_peak", 0.3))
    p.absorb_max = float(cfg.get("absorb_max", 0.0))
    return p


def _stream():
    return _V(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None, numel=None, name="array"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {numel}")
    return _V(t.data_ptr())


def _check(status, where):
    if status != 0:
        raise GicError(status, where)


class Context:
    """A gic_ctx: parameters, sort scratch and the latched error word."""

    def __init__(self, cfg: dict, n_max: int, precision: str = "fp32", r_max: float = None):
        self.cfg = dict(cfg)
        self.precision = precision
        self.params = make_params(cfg, precision, r_max)
        self.n_max = int(n_max)
        self.real = torch.float32 if precision == "fp32" else torch.float64
        L = lib()
        self.K = int(L.gic_key_space(C.byref(self.params)))
        if self.K < 0:
            raise GicError(1, "gic_key_space")
        self.G = int(cfg["n"][0]) * int(cfg["n"][1]) * int(cfg["n"][2])
        h = _V()
        _check(L.gic_create(C.byref(self.params), self.n_max, C.byref(h)), "gic_create")
        self.handle = h

    def set_params(self, **over):
        for k, val in over.items():
            if k == "g":
                self.params.g = (C.c_double * 3)(*val)
            else:
                setattr(self.params, k, float(val))
            self.cfg[k] = val
        _check(lib().gic_set_params(self.handle, C.byref(self.params)), "gic_set_params")

    def error(self, clear=True):
        code = _I32()
        idx = _I64()
        _check(lib().gic_get_error(self.handle, _stream(), C.byref(code), C.byref(idx), int(clear)),
               "gic_get_error")
        return int(code.value), int(idx.value)

    def neighbour_builds(self):
        """Neighbour-list builds on this context so far (synchronises)."""
        b = _I64()
        _check(lib().gic_neighbour_builds(self.handle, _stream(), C.byref(b)), "gic_neighbour_builds")
        return int(b.value)

    STAGES = ("sort", "gather", "contact", "exchange", "grid_clear", "integrate_p2g", "assemble")

    def stage_timing(self, max_steps):
        """Record stage events in the next max_steps (sub-)steps (0: off)."""
        _check(lib().gic_stage_timing(self.handle, int(max_steps)), "gic_stage_timing")

    def stage_times(self):
        """(dict stage -> summed ms, number of steps) since the last call
        (synchronises)."""
        ms = (C.c_double * 7)()
        k = _I32()
        _check(lib().gic_stage_times(self.handle, _stream(), ms, C.byref(k)), "gic_stage_times")
        return dict(zip(self.STAGES, list(ms))), int(k.value)

    def close(self):
        if getattr(self, "handle", None):
            lib().gic_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gic_sort_cells(ctx, x, key, order, cell_begin, cell_end):
    n = x.shape[-1]
    _check(lib().gic_sort_cells(ctx.handle, n, _ptr(x, torch.float64, 3 * n, "x"), _ptr(key, torch.int32, n, "key"),
                                _ptr(order, torch.int32, n, "order"), _ptr(cell_begin, torch.int32, ctx.K, "cell_begin"),
                                _ptr(cell_end, torch.int32, ctx.K, "cell_end"), _stream()), "gic_sort_cells")


def gic_brick_list(ctx, cell_begin, cell_end):
    """Build and keep the brick schedule of these cell tables for the calls
    that follow (until the next sort or stepping call)."""
    _check(lib().gic_brick_list(ctx.handle, _ptr(cell_begin, torch.int32, ctx.K, "cell_begin"),
                                _ptr(cell_end, torch.int32, ctx.K, "cell_end"), _stream()), "gic_brick_list")


def gic_reorder(ctx, order, x, v, r, id_, x_out, v_out, r_out, id_out):
    n = x.shape[-1]
    f64 = torch.float64
    _check(lib().gic_reorder(ctx.handle, n, _ptr(order, torch.int32, n), _ptr(x, f64, 3 * n), _ptr(v, f64, 3 * n),
                             _ptr(r, f64, n), _ptr(id_, torch.int32, n), _ptr(x_out, f64, 3 * n),
                             _ptr(v_out, f64, 3 * n), _ptr(r_out, f64, n), _ptr(id_out, torch.int32, n), _stream()),
           "gic_reorder")


def gic_contact_forces(ctx, x, v, r, cell_begin, cell_end, f_contact, n_contacts=None, pair_ids=None):
    """pair_ids: optional (cap, n) int32 tensor receiving the touching
    partners of every granule (sorted positions, -1 after the last)."""
    n = x.shape[-1]
    f64 = torch.float64
    cap = 0 if pair_ids is None else pair_ids.numel() // max(n, 1)
    _check(lib().gic_contact_forces(ctx.handle, n, _ptr(x, f64, 3 * n), _ptr(v, f64, 3 * n), _ptr(r, f64, n),
                                    _ptr(cell_begin, torch.int32, ctx.K), _ptr(cell_end, torch.int32, ctx.K),
                                    _ptr(f_contact, ctx.real, 3 * n, "f_contact"),
                                    _ptr(n_contacts, torch.int32, n), _ptr(pair_ids, torch.int32, cap * n, "pair_ids"),
                                    int(cap), _stream()), "gic_contact_forces")


def gic_contact_capillary_forces(ctx, x, v, r, sr, cell_begin, cell_end, f_contact, n_contacts=None, held=None):
    n = x.shape[-1]
    f64 = torch.float64
    _check(lib().gic_contact_capillary_forces(ctx.handle, n, _ptr(x, f64, 3 * n), _ptr(v, f64, 3 * n),
                                              _ptr(r, f64, n), _ptr(sr, ctx.real, n, "sr"), _ptr(held, f64, n, "held"),
                                              _ptr(cell_begin, torch.int32, ctx.K), _ptr(cell_end, torch.int32, ctx.K),
                                              _ptr(f_contact, ctx.real, 3 * n, "f_contact"),
                                              _ptr(n_contacts, torch.int32, n), _stream()),
           "gic_contact_capillary_forces")


def gic_moisture_ratio(ctx, held, alpha_f, sr):
    n = held.shape[-1]
    _check(lib().gic_moisture_ratio(ctx.handle, n, _ptr(held, torch.float64, n, "held"),
                                    _ptr(alpha_f, ctx.real, n, "alpha_f"), _ptr(sr, ctx.real, n, "sr"), _stream()),
           "gic_moisture_ratio")


# ---- density projection (Sec. 5.1, Eq. 12b, 13): grids of G cells, double;
# labels uint8 (0 fluid, 1 air, 2 solid) -------------------------------------

def _faces(ctx):
    n0, n1, n2 = (int(v) for v in ctx.cfg["n"])
    return (n0 + 1) * n1 * n2, n0 * (n1 + 1) * n2, n0 * n1 * (n2 + 1)


def idp_workspace(ctx):
    """A device workspace for gic_idp_solve / gic_density_projection."""
    nbytes = int(lib().gic_idp_workspace_bytes(ctx.handle))
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def gic_idp_setup(ctx, alpha_fx, alpha_star, label, alpha_t, rhs):
    G, f64 = ctx.G, torch.float64
    _check(lib().gic_idp_setup(ctx.handle, _ptr(alpha_fx, torch.int64, G), _ptr(alpha_star, f64, G, "alpha_star"),
                               _ptr(label, torch.uint8, G, "label"), _ptr(alpha_t, f64, G, "alpha_t"),
                               _ptr(rhs, f64, G, "rhs"), _stream()), "gic_idp_setup")


def gic_idp_apply(ctx, alpha_t, label, q, out):
    G, f64 = ctx.G, torch.float64
    _check(lib().gic_idp_apply(ctx.handle, _ptr(alpha_t, f64, G), _ptr(label, torch.uint8, G), _ptr(q, f64, G),
                               _ptr(out, f64, G), _stream()), "gic_idp_apply")


def gic_idp_solve(ctx, alpha_t, label, rhs, q, work, max_iter=2000, tol=1e-8, check_every=32, precond=1):
    """Solves L q = rhs in place (q: initial guess in, solution out);
    returns (iterations, relative residual).  Synchronises."""
    G, f64 = ctx.G, torch.float64
    it, rel = _I32(), C.c_double()
    _check(lib().gic_idp_solve(ctx.handle, _ptr(alpha_t, f64, G), _ptr(label, torch.uint8, G), _ptr(rhs, f64, G),
                               _ptr(q, f64, G), _ptr(work, torch.uint8, int(lib().gic_idp_workspace_bytes(ctx.handle))),
                               int(max_iter), float(tol), int(check_every), int(precond), C.byref(it), C.byref(rel),
                               _stream()), "gic_idp_solve")
    return int(it.value), float(rel.value)


def gic_idp_displacement(ctx, q, label, fx, fy, fz):
    G, f64 = ctx.G, torch.float64
    nfx, nfy, nfz = _faces(ctx)
    _check(lib().gic_idp_displacement(ctx.handle, _ptr(q, f64, G), _ptr(label, torch.uint8, G),
                                      _ptr(fx, f64, nfx, "fx"), _ptr(fy, f64, nfy, "fy"), _ptr(fz, f64, nfz, "fz"),
                                      _stream()), "gic_idp_displacement")


def gic_density_projection(ctx, alpha_fx, alpha_star, label, q, fx, fy, fz, work, max_iter=2000, tol=1e-8,
                           check_every=32, precond=1):
    """The whole projection; returns (iterations, relative residual)."""
    G, f64 = ctx.G, torch.float64
    nfx, nfy, nfz = _faces(ctx)
    it, rel = _I32(), C.c_double()
    _check(lib().gic_density_projection(ctx.handle, _ptr(alpha_fx, torch.int64, G), _ptr(alpha_star, f64, G),
                                        _ptr(label, torch.uint8, G), _ptr(q, f64, G), _ptr(fx, f64, nfx, "fx"),
                                        _ptr(fy, f64, nfy, "fy"), _ptr(fz, f64, nfz, "fz"),
                                        _ptr(work, torch.uint8, int(lib().gic_idp_workspace_bytes(ctx.handle))),
                                        int(max_iter), float(tol), int(check_every), int(precond), C.byref(it),
                                        C.byref(rel), _stream()), "gic_density_projection")
    return int(it.value), float(rel.value)


def gic_g2p(ctx, x, u, alpha_fx, alpha_real, u_at, alpha_f):
    n = x.shape[-1]
    _check(lib().gic_g2p(ctx.handle, n, _ptr(x, torch.float64, 3 * n), _ptr(u, ctx.real, 3 * ctx.G, "u"),
                         _ptr(alpha_fx, torch.int64, ctx.G), _ptr(alpha_real, torch.float64, ctx.G),
                         _ptr(u_at, ctx.real, 3 * n, "u_at"), _ptr(alpha_f, ctx.real, n, "alpha_f"), _stream()),
           "gic_g2p")


def gic_drag(ctx, r, v, u_at, alpha_f, f_drag):
    n = r.shape[-1]
    _check(lib().gic_drag(ctx.handle, n, _ptr(r, torch.float64, n), _ptr(v, torch.float64, 3 * n),
                          _ptr(u_at, ctx.real, 3 * n), _ptr(alpha_f, ctx.real, n), _ptr(f_drag, ctx.real, 3 * n),
                          _stream()), "gic_drag")


def gic_integrate(ctx, r, f_contact, f_drag, x, v):
    n = r.shape[-1]
    _check(lib().gic_integrate(ctx.handle, n, _ptr(r, torch.float64, n), _ptr(f_contact, ctx.real, 3 * n),
                               _ptr(f_drag, ctx.real, 3 * n), _ptr(x, torch.float64, 3 * n),
                               _ptr(v, torch.float64, 3 * n), _stream()), "gic_integrate")


def gic_p2g(ctx, x, v, r, cell_begin, cell_end, alpha_fx, mom_fx, accumulate=False):
    n = x.shape[-1]
    _check(lib().gic_p2g(ctx.handle, n, _ptr(x, torch.float64, 3 * n), _ptr(v, torch.float64, 3 * n),
                         _ptr(r, torch.float64, n), _ptr(cell_begin, torch.int32, ctx.K),
                         _ptr(cell_end, torch.int32, ctx.K), _ptr(alpha_fx, torch.int64, ctx.G),
                         _ptr(mom_fx, torch.int64, 3 * ctx.G), int(bool(accumulate)), _stream()), "gic_p2g")


def gic_p2g_real(ctx, x, v, r, cell_begin, cell_end, alpha, mom, accumulate=False):
    n = x.shape[-1]
    _check(lib().gic_p2g_real(ctx.handle, n, _ptr(x, torch.float64, 3 * n), _ptr(v, torch.float64, 3 * n),
                              _ptr(r, torch.float64, n), _ptr(cell_begin, torch.int32, ctx.K),
                              _ptr(cell_end, torch.int32, ctx.K), _ptr(alpha, torch.float64, ctx.G),
                              _ptr(mom, torch.float64, 3 * ctx.G), int(bool(accumulate)), _stream()),
           "gic_p2g_real")


def gic_gather_g2p_drag(ctx, order, x, v, r, id_, x_out, v_out, r_out, id_out, u, alpha_fx, cell_begin, cell_end,
                        f_drag, u_at=None, alpha_f=None):
    n = x.shape[-1]
    f64 = torch.float64
    _check(lib().gic_gather_g2p_drag(ctx.handle, n, _ptr(order, torch.int32, n), _ptr(x, f64, 3 * n),
                                     _ptr(v, f64, 3 * n), _ptr(r, f64, n), _ptr(id_, torch.int32, n),
                                     _ptr(x_out, f64, 3 * n), _ptr(v_out, f64, 3 * n), _ptr(r_out, f64, n),
                                     _ptr(id_out, torch.int32, n), _ptr(u, ctx.real, 3 * ctx.G),
                                     _ptr(alpha_fx, torch.int64, ctx.G), _ptr(cell_begin, torch.int32, ctx.K),
                                     _ptr(cell_end, torch.int32, ctx.K), _ptr(f_drag, ctx.real, 3 * n, "f_drag"),
                                     _ptr(u_at, ctx.real, 3 * n), _ptr(alpha_f, ctx.real, n), _stream()),
           "gic_gather_g2p_drag")


def gic_integrate_p2g(ctx, x, v, r, f_contact, f_drag, cell_begin, cell_end, alpha_fx, mom_fx, accumulate=False):
    n = x.shape[-1]
    f64 = torch.float64
    _check(lib().gic_integrate_p2g(ctx.handle, n, _ptr(x, f64, 3 * n), _ptr(v, f64, 3 * n), _ptr(r, f64, n),
                                   _ptr(f_contact, ctx.real, 3 * n), _ptr(f_drag, ctx.real, 3 * n),
                                   _ptr(cell_begin, torch.int32, ctx.K), _ptr(cell_end, torch.int32, ctx.K),
                                   _ptr(alpha_fx, torch.int64, ctx.G), _ptr(mom_fx, torch.int64, 3 * ctx.G),
                                   int(bool(accumulate)), _stream()), "gic_integrate_p2g")


def gic_integrate_p2g_wet(ctx, x, v, r, held, f_contact, f_drag, cell_begin, cell_end, alpha_fx, mom_fx,
                          accumulate=False):
    n = x.shape[-1]
    f64 = torch.float64
    _check(lib().gic_integrate_p2g_wet(ctx.handle, n, _ptr(x, f64, 3 * n), _ptr(v, f64, 3 * n), _ptr(r, f64, n),
                                       _ptr(held, f64, n, "held"), _ptr(f_contact, ctx.real, 3 * n),
                                       _ptr(f_drag, ctx.real, 3 * n), _ptr(cell_begin, torch.int32, ctx.K),
                                       _ptr(cell_end, torch.int32, ctx.K), _ptr(alpha_fx, torch.int64, ctx.G),
                                       _ptr(mom_fx, torch.int64, 3 * ctx.G), int(bool(accumulate)), _stream()),
           "gic_integrate_p2g_wet")


def gic_step(ctx, cur, nxt, u, alpha_fx, mom_fx, scratch):
    """One sub-step; cur/nxt: dicts of x, v, r, id tensors; scratch: dict of
    key, order, cell_begin, cell_end, f_contact, f_drag and, optionally,
    u_at, alpha_f (written when present)."""
    n = cur["x"].shape[-1]
    f64 = torch.float64
    s = scratch
    _check(lib().gic_step(ctx.handle, n, _ptr(cur["x"], f64, 3 * n), _ptr(cur["v"], f64, 3 * n),
                          _ptr(cur["r"], f64, n), _ptr(cur.get("id"), torch.int32, n), _ptr(nxt["x"], f64, 3 * n),
                          _ptr(nxt["v"], f64, 3 * n), _ptr(nxt["r"], f64, n), _ptr(nxt.get("id"), torch.int32, n),
                          _ptr(u, ctx.real, 3 * ctx.G), _ptr(alpha_fx, torch.int64, ctx.G),
                          _ptr(mom_fx, torch.int64, 3 * ctx.G), _ptr(s["key"], torch.int32, n),
                          _ptr(s["order"], torch.int32, n), _ptr(s["cell_begin"], torch.int32, ctx.K),
                          _ptr(s["cell_end"], torch.int32, ctx.K), _ptr(s["f_contact"], ctx.real, 3 * n),
                          _ptr(s["f_drag"], ctx.real, 3 * n), _ptr(s.get("u_at"), ctx.real, 3 * n),
                          _ptr(s.get("alpha_f"), ctx.real, n), _stream()), "gic_step")


# ---- remaining interphase forces and the sand step ------------------------------

def gic_gather_g2p_fluid(ctx, order, x, v, r, id_, x_out, v_out, r_out, id_out, u, alpha_fx, cell_begin, cell_end,
                         f_fluid, grad_p=None, acc_f=None, held=None, held_out=None):
    n = x.shape[-1]
    f64 = torch.float64
    _check(lib().gic_gather_g2p_fluid(ctx.handle, n, _ptr(order, torch.int32, n), _ptr(x, f64, 3 * n),
                                      _ptr(v, f64, 3 * n), _ptr(r, f64, n), _ptr(id_, torch.int32, n),
                                      _ptr(x_out, f64, 3 * n), _ptr(v_out, f64, 3 * n), _ptr(r_out, f64, n),
                                      _ptr(id_out, torch.int32, n), _ptr(u, ctx.real, 3 * ctx.G),
                                      _ptr(alpha_fx, torch.int64, ctx.G), _ptr(grad_p, ctx.real, 3 * ctx.G),
                                      _ptr(acc_f, ctx.real, 3 * ctx.G), _ptr(cell_begin, torch.int32, ctx.K),
                                      _ptr(cell_end, torch.int32, ctx.K), _ptr(f_fluid, ctx.real, 3 * n, "f_fluid"),
                                      _ptr(held, f64, n, "held"), _ptr(held_out, f64, n, "held_out"), _stream()),
           "gic_gather_g2p_fluid")


def gic_exchange_p2g(ctx, x, r, f_contact, f_fluid, cell_begin, cell_end, weight, fs_fx, held=None):
    n = x.shape[-1]
    f64 = torch.float64
    _check(lib().gic_exchange_p2g(ctx.handle, n, _ptr(x, f64, 3 * n), _ptr(r, f64, n),
                                  _ptr(f_contact, ctx.real, 3 * n), _ptr(f_fluid, ctx.real, 3 * n),
                                  _ptr(cell_begin, torch.int32, ctx.K), _ptr(cell_end, torch.int32, ctx.K),
                                  float(weight), _ptr(fs_fx, torch.int64, 3 * ctx.G), _ptr(held, f64, n, "held"),
                                  _stream()), "gic_exchange_p2g")


def gic_sand_step(ctx, a, b, Dt, u, alpha_fx, mom_fx, scratch, grad_p=None, acc_f=None, fs_fx=None):
    """One sand step of length Dt in ceil(Dt / dt) sub-steps; a, b: dicts of
    x, v, r, id tensors (the state starts in a).  Returns (N, which): the
    number of sub-steps and 0 if the state ends in a, 1 if in b.  scratch:
    key, order, cell_begin, cell_end, f_contact, f_drag (the fluid force)."""
    n = a["x"].shape[-1]
    f64 = torch.float64
    s = scratch
    N = C.c_int32(0)
    which = C.c_int32(0)
    _check(lib().gic_sand_step(ctx.handle, n, float(Dt), _ptr(a["x"], f64, 3 * n), _ptr(a["v"], f64, 3 * n),
                               _ptr(a["r"], f64, n), _ptr(a.get("id"), torch.int32, n), _ptr(b["x"], f64, 3 * n),
                               _ptr(b["v"], f64, 3 * n), _ptr(b["r"], f64, n), _ptr(b.get("id"), torch.int32, n),
                               _ptr(u, ctx.real, 3 * ctx.G), _ptr(grad_p, ctx.real, 3 * ctx.G),
                               _ptr(acc_f, ctx.real, 3 * ctx.G), _ptr(alpha_fx, torch.int64, ctx.G),
                               _ptr(mom_fx, torch.int64, 3 * ctx.G), _ptr(fs_fx, torch.int64, 3 * ctx.G),
                               _ptr(s["key"], torch.int32, n), _ptr(s["order"], torch.int32, n),
                               _ptr(s["cell_begin"], torch.int32, ctx.K), _ptr(s["cell_end"], torch.int32, ctx.K),
                               _ptr(s["f_contact"], ctx.real, 3 * n), _ptr(s["f_drag"], ctx.real, 3 * n),
                               C.byref(N), C.byref(which), _stream()), "gic_sand_step")
    return int(N.value), int(which.value)


# ---- adjoint form (double) ----------------------------------------------------

def gic_contact_forces_vjp(ctx, x, v, r, cell_begin, cell_end, g_f, g_x, g_v, g_mu):
    n = x.shape[-1]
    f64 = torch.float64
    _check(lib().gic_contact_forces_vjp(ctx.handle, n, _ptr(x, f64, 3 * n), _ptr(v, f64, 3 * n), _ptr(r, f64, n),
                                        _ptr(cell_begin, torch.int32, ctx.K), _ptr(cell_end, torch.int32, ctx.K),
                                        _ptr(g_f, f64, 3 * n), _ptr(g_x, f64, 3 * n), _ptr(g_v, f64, 3 * n),
                                        _ptr(g_mu, f64, n), _stream()), "gic_contact_forces_vjp")


def gic_drag_vjp(ctx, r, v, u_at, alpha_f, g_f, g_v, g_u_at, g_alpha_f, g_cdrag):
    n = r.shape[-1]
    f64 = torch.float64
    _check(lib().gic_drag_vjp(ctx.handle, n, _ptr(r, f64, n), _ptr(v, f64, 3 * n), _ptr(u_at, f64, 3 * n),
                              _ptr(alpha_f, f64, n), _ptr(g_f, f64, 3 * n), _ptr(g_v, f64, 3 * n),
                              _ptr(g_u_at, f64, 3 * n), _ptr(g_alpha_f, f64, n), _ptr(g_cdrag, f64, n), _stream()),
           "gic_drag_vjp")


def gic_integrate_vjp(ctx, r, g_x, g_v, g_f):
    n = r.shape[-1]
    f64 = torch.float64
    _check(lib().gic_integrate_vjp(ctx.handle, n, _ptr(r, f64, n), _ptr(g_x, f64, 3 * n), _ptr(g_v, f64, 3 * n),
                                   _ptr(g_f, f64, 3 * n), _stream()), "gic_integrate_vjp")


def gic_g2p_vjp(ctx, x, u, alpha_real, g_u_at, g_alpha_f, cell_begin, cell_end, g_x, g_alpha):
    n = x.shape[-1]
    f64 = torch.float64
    _check(lib().gic_g2p_vjp(ctx.handle, n, _ptr(x, f64, 3 * n), _ptr(u, f64, 3 * ctx.G),
                             _ptr(alpha_real, f64, ctx.G), _ptr(g_u_at, f64, 3 * n), _ptr(g_alpha_f, f64, n),
                             _ptr(cell_begin, torch.int32, ctx.K), _ptr(cell_end, torch.int32, ctx.K),
                             _ptr(g_x, f64, 3 * n), _ptr(g_alpha, f64, ctx.G), _stream()), "gic_g2p_vjp")


def gic_p2g_vjp(ctx, x, v, r, g_alpha, g_mom, g_x, g_v):
    n = x.shape[-1]
    f64 = torch.float64
    _check(lib().gic_p2g_vjp(ctx.handle, n, _ptr(x, f64, 3 * n), _ptr(v, f64, 3 * n), _ptr(r, f64, n),
                             _ptr(g_alpha, f64, ctx.G), _ptr(g_mom, f64, 3 * ctx.G), _ptr(g_x, f64, 3 * n),
                             _ptr(g_v, f64, 3 * n), _stream()), "gic_p2g_vjp")


def gic_sum(ctx, a, out, b=None, accumulate=False):
    _check(lib().gic_sum(ctx.handle, a.numel(), _ptr(a, torch.float64), _ptr(b, torch.float64, a.numel()),
                         _ptr(out, torch.float64, 1), int(bool(accumulate)), _stream()), "gic_sum")


def gic_sum_noalloc(a, out, b=None, accumulate=False):
    """gic_sum without a context: its partial sums live in a fixed array
    that the library holds on each device (no allocation in the call)."""
    _check(lib().gic_sum_noalloc(a.numel(), _ptr(a, torch.float64), _ptr(b, torch.float64, a.numel()),
                                 _ptr(out, torch.float64, 1), int(bool(accumulate)), _stream()), "gic_sum_noalloc")


def gic_scale(ctx, a, s, factor, out):
    """out = (factor s[0]) a, s a one-element device tensor (float64)."""
    n = a.numel()
    _check(lib().gic_scale(ctx.handle, n, _ptr(a, torch.float64), _ptr(s, torch.float64, 1, "s"), float(factor),
                           _ptr(out, torch.float64, n, "out"), _stream()), "gic_scale")


def gic_permute(ctx, order, src, dst, comps, scatter):
    n = order.numel()
    _check(lib().gic_permute(ctx.handle, n, int(comps), _ptr(order, torch.int32, n),
                             _ptr(src, torch.float64, comps * n), _ptr(dst, torch.float64, comps * n),
                             int(bool(scatter)), _stream()), "gic_permute")


class Simulator:
    """Granule state on the GPU plus the buffers of one sub-step.

    The state (x, v, r, id) is double-buffered: each step reads `cur` and
    writes the advanced state, in the new sorted order, to `nxt`, then swaps.
    id[q] is the input index of the granule now at position q."""

    def __init__(self, cfg, x, v, r, u, precision="fp32", r_max=None, device="cuda"):
        n = x.shape[-1]
        self.n = n
        self.ctx = Context(cfg, n, precision, r_max)
        dev = torch.device(device)
        f64 = torch.float64
        real = self.ctx.real
        self.cur = dict(x=torch.as_tensor(x, dtype=f64).to(dev).contiguous(),
                        v=torch.as_tensor(v, dtype=f64).to(dev).contiguous(),
                        r=torch.as_tensor(r, dtype=f64).to(dev).contiguous(),
                        id=torch.arange(n, dtype=torch.int32, device=dev))
        self.nxt = {k: torch.empty_like(t) for k, t in self.cur.items()}
        self.u = torch.as_tensor(u).to(dev, real).contiguous()
        G, K = self.ctx.G, self.ctx.K
        self.alpha = torch.zeros(G, dtype=torch.int64, device=dev)
        self.mom = torch.zeros(3 * G, dtype=torch.int64, device=dev)
        self.scratch = dict(key=torch.empty(n, dtype=torch.int32, device=dev),
                            order=torch.empty(n, dtype=torch.int32, device=dev),
                            cell_begin=torch.empty(K, dtype=torch.int32, device=dev),
                            cell_end=torch.empty(K, dtype=torch.int32, device=dev),
                            f_contact=torch.empty(3 * n, dtype=real, device=dev),
                            f_drag=torch.empty(3 * n, dtype=real, device=dev),
                            u_at=torch.empty(3 * n, dtype=real, device=dev),
                            alpha_f=torch.empty(n, dtype=real, device=dev))
        # the step itself does not need the sampled fluid velocity and fraction
        self.step_scratch = {k: t for k, t in self.scratch.items() if k not in ("u_at", "alpha_f")}
        self.init_grid()

    def init_grid(self):
        """alpha, momentum = P2G of the current state (Alg. 1 initial state)."""
        s = self.scratch
        gic_sort_cells(self.ctx, self.cur["x"], s["key"], s["order"], s["cell_begin"], s["cell_end"])
        gic_reorder(self.ctx, s["order"], self.cur["x"], self.cur["v"], self.cur["r"], self.cur["id"],
                    self.nxt["x"], self.nxt["v"], self.nxt["r"], self.nxt["id"])
        self.cur, self.nxt = self.nxt, self.cur
        gic_p2g(self.ctx, self.cur["x"], self.cur["v"], self.cur["r"], s["cell_begin"], s["cell_end"], self.alpha,
                self.mom)

    def step(self, k=1):
        for _ in range(k):
            gic_step(self.ctx, self.cur, self.nxt, self.u, self.alpha, self.mom, self.step_scratch)
            self.cur, self.nxt = self.nxt, self.cur

    def sand_step(self, Dt, grad_p=None, acc_f=None, fs=None):
        """One sand step of length Dt (Alg. 2) with frozen fluid fields;
        grad_p, acc_f: (3G) real tensors or None; fs: (3G) int64 exchange grid
        (accumulated) or None.  Returns the number of sub-steps."""
        N, which = gic_sand_step(self.ctx, self.cur, self.nxt, Dt, self.u, self.alpha, self.mom, self.step_scratch,
                                 grad_p=grad_p, acc_f=acc_f, fs_fx=fs)
        if which:
            self.cur, self.nxt = self.nxt, self.cur
        return N

    def state_in_input_order(self):
        """(x, v) as (3, n) float64 CPU arrays indexed by input granule."""
        idx = self.cur["id"].long()
        x = torch.empty_like(self.cur["x"]).view(3, -1)
        v = torch.empty_like(self.cur["v"]).view(3, -1)
        x[:, idx] = self.cur["x"].view(3, -1)
        v[:, idx] = self.cur["v"].view(3, -1)
        return x.cpu().numpy(), v.cpu().numpy()
