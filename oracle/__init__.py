"""FP64 CPU oracle of the Granule-In-Cell granule step -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding) never
imports it.

Thin ctypes wrapper over oracle.c: numpy arrays in, numpy arrays out.  Each
wrapper names the passage of the paper its C function follows.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class OrcParams(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3), ("dx", C.c_double), ("nc", C.c_int32 * 3), ("cell", C.c_double),
        ("kn", C.c_double), ("restitution", C.c_double), ("kt_ratio", C.c_double), ("mu", C.c_double),
        ("rho_s", C.c_double), ("eta_f", C.c_double), ("c_drag", C.c_double), ("alpha_max", C.c_double),
        ("g", C.c_double * 3), ("dt", C.c_double), ("walls", C.c_uint32), ("pad", C.c_int32),
        ("absorb_max", C.c_double),
    ]


def params(cfg: dict) -> OrcParams:
    """Oracle parameter block from a workload parameter dict."""
    p = OrcParams()
    p.n = (C.c_int32 * 3)(*cfg["n"])
    p.dx = cfg["dx"]
    p.nc = (C.c_int32 * 3)(*cfg["nc"])
    p.cell = cfg["cell"]
    for k in ("kn", "restitution", "kt_ratio", "mu", "rho_s", "eta_f", "c_drag", "alpha_max", "dt"):
        setattr(p, k, float(cfg[k]))
    p.g = (C.c_double * 3)(*cfg["g"])
    p.walls = int(cfg["walls"])
    # maximum absorption ratio of Sec. 5.3: raises the alpha_s clamp (0: dry)
    p.absorb_max = float(cfg.get("absorb_max", 0.0))
    return p


class OrcCoupling(C.Structure):
    _fields_ = [
        ("rho_f", C.c_double), ("c_quad", C.c_double), ("f_unit", C.c_double),
        ("drag_model", C.c_int32), ("vmass", C.c_int32),
    ]


def coupling(cfg: dict) -> OrcCoupling:
    """Oracle parameters of the remaining interphase forces from a workload
    parameter dict (absent keys: linear drag only, no virtual mass)."""
    c = OrcCoupling()
    c.rho_f = float(cfg.get("rho_f", 0.0))
    c.c_quad = float(cfg.get("c_quad", 0.0))
    c.f_unit = float(cfg.get("f_unit", 1.0))
    c.drag_model = int(cfg.get("drag_model", 0))
    c.vmass = int(cfg.get("vmass", 0))
    return c


class OrcCapillary(C.Structure):
    _fields_ = [("sigma", C.c_double), ("vbridge", C.c_double), ("sr_peak", C.c_double)]


def capillary(cfg: dict) -> OrcCapillary:
    """Oracle parameters of the capillary pair force (absent keys: off)."""
    c = OrcCapillary()
    c.sigma = float(cfg.get("sigma", 0.0))
    c.vbridge = float(cfg.get("vbridge", 1e-4))
    c.sr_peak = float(cfg.get("sr_peak", 0.3))
    return c


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        _LIB = C.CDLL(path)
        _declare(_LIB)
    return _LIB


_P = C.POINTER
_d = _P(C.c_double)
_i64 = _P(C.c_int64)
_i32 = _P(C.c_int32)
_u32 = _P(C.c_uint32)
_pp = _P(OrcParams)
_pc = _P(OrcCoupling)
_pk = _P(OrcCapillary)


def _declare(L):
    sig = {
        "orc_key_space": (C.c_int64, [_pp]),
        "orc_cell_keys": (None, [_pp, C.c_int64, _d, _u32]),
        "orc_stable_sort": (None, [C.c_int64, _u32, _i32]),
        "orc_cell_ranges": (None, [_pp, C.c_int64, _u32, _i32, _i32, _i32]),
        "orc_pairs_brute": (C.c_int64, [C.c_int64, _d, _d, C.c_int64, _i32, _i32]),
        "orc_pairs_cells": (C.c_int64, [_pp, C.c_int64, _d, _d, C.c_int64, _i32, _i32]),
        "orc_pairs_sample": (None, [_pp, C.c_int64, _d, _d, C.c_int64, _i64, C.c_int64, _i32, _i32]),
        "orc_contact_forces": (None, [_pp, C.c_int64, _d, _d, _d, _d, _d, _i32, _i32]),
        "orc_contact_forces_sample": (None, [_pp, C.c_int64, _d, _d, _d, C.c_int64, _i64, _d, _d]),
        "orc_pair": (C.c_int, [_pp, _d, _d, _d, _d, C.c_double, C.c_double, _d, _i32]),
        "orc_stencil27": (None, [_pp, _d, _d, _i64, _d]),
        "orc_p2g_fixed": (None, [_pp, C.c_int64, _d, _d, _d, _i64, _i64]),
        "orc_round_product_x": (C.c_int64, [C.c_double, C.c_double]),
        "orc_p2g_totals_x": (None, [_pp, C.c_double, _d, _d]),
        "orc_p2g_real": (None, [_pp, C.c_int64, _d, _d, _d, _d, _d]),
        "orc_g2p": (None, [_pp, C.c_int64, _d, _d, _i64, _d, _d, _d]),
        "orc_drag": (None, [_pp, C.c_int64, _d, _d, _d, _d, _d]),
        "orc_integrate": (None, [_pp, C.c_int64, _d, _d, _d, _d, _d]),
        "orc_step": (None, [_pp, C.c_int64, _d, _d, _d, _d, _i64, _i64, _d, _d, _d, _d]),
        "orc_contact_vjp": (None, [_pp, C.c_int64, _d, _d, _d, _d, _d, _d, _d]),
        "orc_drag_vjp": (None, [_pp, C.c_int64, _d, _d, _d, _d, _d, _d, _d, _d, _d]),
        "orc_g2p_vjp": (None, [_pp, C.c_int64, _d, _d, _d, _d, _d, _d, _d]),
        "orc_p2g_vjp": (None, [_pp, C.c_int64, _d, _d, _d, _d, _d, _d, _d]),
        "orc_rollout": (C.c_double, [_pp, C.c_int64, _d, _d, _d, _d, C.c_int32, _d, _P(C.c_uint64)]),
        "orc_rollout_vjp": (C.c_double, [_pp, C.c_int64, _d, _d, _d, _d, C.c_int32, _d, _d, _d]),
        "orc_fluid_forces": (None, [_pp, _pc, C.c_int64, _d, _d, _d, _d, _d, _i64, _d, _d, _d]),
        "orc_integrate_vm": (None, [_pp, _pc, C.c_int64, _d, _d, _d, _d, _d]),
        "orc_exchange_force": (None, [_pp, _pc, C.c_int64, _d, _d, _d, _d, _d]),
        "orc_exchange_p2g": (None, [_pp, _pc, C.c_int64, _d, _d, _d, _d, _d, C.c_double, _i64]),
        "orc_substeps": (C.c_int32, [C.c_double, C.c_double]),
        "orc_sand_step": (C.c_int32, [_pp, _pc, C.c_int64, C.c_double, _d, _d, _d, _d, _d, _d, _i64, _i64, _i64]),
        "orc_gamma": (C.c_double, [_pk, C.c_double]),
        "orc_moisture_ratio": (None, [C.c_int64, _d, _d, _d]),
        "orc_wet_mass": (None, [_pp, C.c_double, C.c_int64, _d, _d, _d]),
        "orc_contact_forces_wet": (None, [_pp, C.c_int64, _d, _d, _d, _d, _d, _d, _P(C.c_int32)]),
        "orc_contact_forces_sample_wet": (None, [_pp, C.c_int64, _d, _d, _d, _d, C.c_int64, _i64, _d, _d]),
        "orc_integrate_wet": (None, [_pp, _pc, C.c_int64, _d, _d, _d, _d, _d, _d, _d]),
        "orc_p2g_fixed_wet": (None, [_pp, C.c_double, C.c_int64, _d, _d, _d, _d, _i64, _i64]),
        "orc_bridge": (None, [_pk, C.c_double, _d, _d]),
        "orc_bridge_energy": (C.c_double, [_pk, C.c_double, C.c_double]),
        "orc_fst": (C.c_double, [_pk, C.c_double, C.c_double]),
        "orc_capillary_pair_force": (None, [_pk, _d, _d, C.c_double, C.c_double, C.c_double, C.c_double, _d]),
        "orc_capillary_forces": (None, [_pp, _pk, C.c_int64, _d, _d, _d, _d]),
        "orc_capillary_forces_sample": (None, [_pp, _pk, C.c_int64, _d, _d, _d, C.c_int64, _i64, _d, _d]),
        "orc_num_threads": (C.c_int, []),
        "orc_set_num_threads": (None, [C.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(_P(ctype))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def nodes(cfg):
    n = cfg["n"]
    return int(n[0]) * int(n[1]) * int(n[2])


def key_space(cfg):
    p = params(cfg)
    return int(lib().orc_key_space(C.byref(p)))


def num_threads():
    return int(lib().orc_num_threads())


def set_num_threads(t):
    lib().orc_set_num_threads(int(t))


# ---- binning / neighbour search (support of Sec. 3.1's contact test) --------

def cell_keys(cfg, x):
    """Brick-major neighbour-cell key per granule (uint32)."""
    x = _f64(x)
    n = x.shape[1]
    key = np.zeros(n, np.uint32)
    p = params(cfg)
    lib().orc_cell_keys(C.byref(p), n, _ptr(x, C.c_double), _ptr(key, C.c_uint32))
    return key


def stable_sort(key):
    key = np.ascontiguousarray(key, np.uint32)
    order = np.zeros(key.shape[0], np.int32)
    lib().orc_stable_sort(key.shape[0], _ptr(key, C.c_uint32), _ptr(order, C.c_int32))
    return order


def cell_ranges(cfg, key, order):
    key = np.ascontiguousarray(key, np.uint32)
    order = np.ascontiguousarray(order, np.int32)
    K = key_space(cfg)
    begin = np.zeros(K, np.int32)
    end = np.zeros(K, np.int32)
    p = params(cfg)
    lib().orc_cell_ranges(C.byref(p), key.shape[0], _ptr(key, C.c_uint32), _ptr(order, C.c_int32),
                          _ptr(begin, C.c_int32), _ptr(end, C.c_int32))
    return begin, end


def _pairs(fn, args, n_guess):
    cap = max(16, n_guess)
    while True:
        pi = np.zeros(cap, np.int32)
        pj = np.zeros(cap, np.int32)
        cnt = fn(*args, cap, _ptr(pi, C.c_int32), _ptr(pj, C.c_int32))
        if cnt <= cap:
            return np.stack([pi[:cnt], pj[:cnt]], 1)
        cap = int(cnt)


def pairs_brute(x, r):
    """Touching pairs (i < j) by the O(N^2) definition d_ij < r_i + r_j (Sec. 3.1)."""
    x = _f64(x)
    r = _f64(r)
    return _pairs(lib().orc_pairs_brute, (x.shape[1], _ptr(x, C.c_double), _ptr(r, C.c_double)), 8 * x.shape[1])


def pairs_cells(cfg, x, r):
    """The same pair set found through the cell list."""
    x = _f64(x)
    r = _f64(r)
    p = params(cfg)
    return _pairs(lib().orc_pairs_cells,
                  (C.byref(p), x.shape[1], _ptr(x, C.c_double), _ptr(r, C.c_double)), 8 * x.shape[1])


def pairs_sample(cfg, x, r, idx, cap=64):
    """Touching partners of the sampled granules idx: a list of sets."""
    x, r = _f64(x), _f64(r)
    idx = np.ascontiguousarray(idx, np.int64)
    m = idx.shape[0]
    part = np.zeros(m * cap, np.int32)
    cnt = np.zeros(m, np.int32)
    lib().orc_pairs_sample(C.byref(params(cfg)), x.shape[1], _ptr(x, C.c_double), _ptr(r, C.c_double), m,
                           _ptr(idx, C.c_int64), cap, _ptr(part, C.c_int32), _ptr(cnt, C.c_int32))
    assert cnt.max(initial=0) <= cap
    return [set(part[s * cap:s * cap + cnt[s]].tolist()) for s in range(m)]


# ---- contact force, Eq. (1a)-(1c) --------------------------------------------

def contact_forces(cfg, x, v, r):
    """Returns (F (3,n), fabs (n), ncontacts (n), nsliding (n))."""
    x, v, r = _f64(x), _f64(v), _f64(r)
    n = x.shape[1]
    F = np.zeros((3, n))
    fa = np.zeros(n)
    nc = np.zeros(n, np.int32)
    ns = np.zeros(n, np.int32)
    p = params(cfg)
    lib().orc_contact_forces(C.byref(p), n, _ptr(x, C.c_double), _ptr(v, C.c_double), _ptr(r, C.c_double),
                             _ptr(F, C.c_double), _ptr(fa, C.c_double), _ptr(nc, C.c_int32), _ptr(ns, C.c_int32))
    return F, fa, nc, ns


def contact_forces_sample(cfg, x, v, r, idx):
    x, v, r = _f64(x), _f64(v), _f64(r)
    idx = np.ascontiguousarray(idx, np.int64)
    m = idx.shape[0]
    F = np.zeros((3, m))
    fa = np.zeros(m)
    p = params(cfg)
    lib().orc_contact_forces_sample(C.byref(p), x.shape[1], _ptr(x, C.c_double), _ptr(v, C.c_double),
                                    _ptr(r, C.c_double), m, _ptr(idx, C.c_int64), _ptr(F, C.c_double),
                                    _ptr(fa, C.c_double))
    return F, fa


def pair_force(cfg, xi, xj, vi, vj, ri, rj):
    """Force on i from j; returns (F (3,), touching, sliding)."""
    p = params(cfg)
    F = np.zeros(3)
    s = np.zeros(1, np.int32)
    a = [_f64(t) for t in (xi, xj, vi, vj)]
    hit = lib().orc_pair(C.byref(p), *[_ptr(t, C.c_double) for t in a], float(ri), float(rj),
                         _ptr(F, C.c_double), _ptr(s, C.c_int32))
    return F, bool(hit), bool(s[0])


# ---- transfers, Eq. (7a) and the G2P of Sec. 5.2 -----------------------------

def stencil27(cfg, xa):
    p = params(cfg)
    xa = _f64(xa)
    w = np.zeros(27)
    node = np.zeros(27, np.int64)
    w1 = np.zeros(9)
    lib().orc_stencil27(C.byref(p), _ptr(xa, C.c_double), _ptr(w, C.c_double), _ptr(node, C.c_int64),
                        _ptr(w1, C.c_double))
    return w, node, w1.reshape(3, 3)


def p2g_fixed(cfg, x, v, r):
    """(alpha (G,) int64, mom (3,G) int64) in 2^-32 units."""
    x, v, r = _f64(x), _f64(v), _f64(r)
    G = nodes(cfg)
    alpha = np.zeros(G, np.int64)
    mom = np.zeros((3, G), np.int64)
    p = params(cfg)
    lib().orc_p2g_fixed(C.byref(p), x.shape[1], _ptr(x, C.c_double), _ptr(v, C.c_double), _ptr(r, C.c_double),
                        _ptr(alpha, C.c_int64), _ptr(mom, C.c_int64))
    return alpha, mom


def round_product(a, b):
    """The integer a fixed-point contribution a b is rounded to: the exact
    product, rounded once to the nearest integer (ties to even)."""
    return int(lib().orc_round_product_x(float(a), float(b)))


def p2g_totals(cfg, r, va):
    """Scaled totals S (fraction, three momentum channels) of one dry
    granule of radius r and velocity va (3,)."""
    S = np.zeros(4)
    lib().orc_p2g_totals_x(C.byref(params(cfg)), float(r), _ptr(_f64(va), C.c_double), _ptr(S, C.c_double))
    return S


def p2g_real(cfg, x, v, r):
    """(alpha (G,) cell volumes, mom (3,G) kg m/s), unquantised."""
    x, v, r = _f64(x), _f64(v), _f64(r)
    G = nodes(cfg)
    alpha = np.zeros(G)
    mom = np.zeros((3, G))
    p = params(cfg)
    lib().orc_p2g_real(C.byref(p), x.shape[1], _ptr(x, C.c_double), _ptr(v, C.c_double), _ptr(r, C.c_double),
                       _ptr(alpha, C.c_double), _ptr(mom, C.c_double))
    return alpha, mom


def g2p(cfg, x, u, alpha_fx=None, alpha_real=None):
    """(u_at (3,n), alpha_f (n,))."""
    assert (alpha_fx is None) != (alpha_real is None)
    x, u = _f64(x), _f64(u)
    n = x.shape[1]
    uat = np.zeros((3, n))
    af = np.zeros(n)
    afx = None if alpha_fx is None else np.ascontiguousarray(alpha_fx, np.int64)
    are = None if alpha_real is None else _f64(alpha_real)
    p = params(cfg)
    lib().orc_g2p(C.byref(p), n, _ptr(x, C.c_double), _ptr(u, C.c_double), _ptr(afx, C.c_int64),
                  _ptr(are, C.c_double), _ptr(uat, C.c_double), _ptr(af, C.c_double))
    return uat, af


def drag(cfg, r, v, u_at, alpha_f):
    r, v, u_at, alpha_f = _f64(r), _f64(v), _f64(u_at), _f64(alpha_f)
    n = r.shape[0]
    Fd = np.zeros((3, n))
    p = params(cfg)
    lib().orc_drag(C.byref(p), n, _ptr(r, C.c_double), _ptr(v, C.c_double), _ptr(u_at, C.c_double),
                   _ptr(alpha_f, C.c_double), _ptr(Fd, C.c_double))
    return Fd


def integrate(cfg, r, Fc, Fd, x, v):
    """Returns new (x, v); inputs are not modified."""
    r, Fc, Fd = _f64(r), _f64(Fc), _f64(Fd)
    x = _f64(x).copy()
    v = _f64(v).copy()
    p = params(cfg)
    lib().orc_integrate(C.byref(p), r.shape[0], _ptr(r, C.c_double), _ptr(Fc, C.c_double), _ptr(Fd, C.c_double),
                        _ptr(x, C.c_double), _ptr(v, C.c_double))
    return x, v


def step(cfg, x, v, r, u, alpha_fx):
    """One granule step (Alg. 2, one sub-step).  Returns a dict with the new
    x, v, the new alpha / momentum grids and the intermediates."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    r, u = _f64(r), _f64(u)
    n = x.shape[1]
    G = nodes(cfg)
    alpha = np.ascontiguousarray(alpha_fx, np.int64).copy()
    mom = np.zeros((3, G), np.int64)
    Fc = np.zeros((3, n))
    Fd = np.zeros((3, n))
    uat = np.zeros((3, n))
    af = np.zeros(n)
    p = params(cfg)
    lib().orc_step(C.byref(p), n, _ptr(x, C.c_double), _ptr(v, C.c_double), _ptr(r, C.c_double),
                   _ptr(u, C.c_double), _ptr(alpha, C.c_int64), _ptr(mom, C.c_int64), _ptr(Fc, C.c_double),
                   _ptr(Fd, C.c_double), _ptr(uat, C.c_double), _ptr(af, C.c_double))
    return dict(x=x, v=v, alpha=alpha, mom=mom, Fc=Fc, Fd=Fd, u_at=uat, alpha_f=af)


# ---- remaining interphase forces (Sec. 3.3 Eq. 5a-5c, Sec. 5.2 Eq. 9) and the
# ---- full sand step with the exchange momentum (Alg. 2, Sec. 5.2) -----------

def fluid_forces(cfg, x, v, r, u, alpha_fx, gp=None, af=None, held=None):
    """Fluid force on each granule (3,n): drag (cfg drag_model: 0 linear Stokes
    form x alpha_f, 1 quadratic Eq. 5b) + pressure gradient -V grad p (if gp)
    + (1/2) rho_f V dv_f/dt (if vmass and af); gp, af are (3,G) grid fields.
    held (n,): absorbed water per granule volume, extra volume V held in the
    volume forces (Sec. 5.3); None for dry granules."""
    x, v, r, u = _f64(x), _f64(v), _f64(r), _f64(u)
    held = None if held is None else _f64(held)
    n = x.shape[1]
    Ffl = np.zeros((3, n))
    afx = np.ascontiguousarray(alpha_fx, np.int64)
    gp = None if gp is None else _f64(gp)
    af = None if af is None else _f64(af)
    p, c = params(cfg), coupling(cfg)
    lib().orc_fluid_forces(C.byref(p), C.byref(c), n, _ptr(x, C.c_double), _ptr(v, C.c_double),
                           _ptr(r, C.c_double), _ptr(held, C.c_double), _ptr(u, C.c_double), _ptr(afx, C.c_int64),
                           _ptr(gp, C.c_double), _ptr(af, C.c_double), _ptr(Ffl, C.c_double))
    return Ffl


def integrate_vm(cfg, r, Fc, Ffl, x, v):
    """Semi-implicit Euler with the effective mass m + (1/2) rho_f V of Eq. 9
    (plain integrate when cfg vmass is 0).  Returns new (x, v)."""
    r, Fc, Ffl = _f64(r), _f64(Fc), _f64(Ffl)
    x = _f64(x).copy()
    v = _f64(v).copy()
    p, c = params(cfg), coupling(cfg)
    lib().orc_integrate_vm(C.byref(p), C.byref(c), r.shape[0], _ptr(r, C.c_double), _ptr(Fc, C.c_double),
                           _ptr(Ffl, C.c_double), _ptr(x, C.c_double), _ptr(v, C.c_double))
    return x, v


def exchange_force(cfg, r, Fc, Ffl, held=None):
    """Whole fluid force of a sub-step on each granule (3,n); held: wet
    granules (wet mass and volume, Sec. 5.3) or None."""
    r, Fc, Ffl = _f64(r), _f64(Fc), _f64(Ffl)
    held = None if held is None else _f64(held)
    fex = np.zeros_like(Ffl)
    p, c = params(cfg), coupling(cfg)
    lib().orc_exchange_force(C.byref(p), C.byref(c), r.shape[0], _ptr(r, C.c_double), _ptr(held, C.c_double),
                             _ptr(Fc, C.c_double), _ptr(Ffl, C.c_double), _ptr(fex, C.c_double))
    return fex


def exchange_p2g(cfg, x, r, Fc, Ffl, weight, fs=None, held=None):
    """Exchange deposit of one sub-step: fs (3,G) int64 in 2^-32 f_unit units
    accumulates -weight * f_j N(x_j - x)."""
    x, r, Fc, Ffl = _f64(x), _f64(r), _f64(Fc), _f64(Ffl)
    held = None if held is None else _f64(held)
    G = nodes(cfg)
    fs = np.zeros((3, G), np.int64) if fs is None else np.ascontiguousarray(fs, np.int64).copy()
    p, c = params(cfg), coupling(cfg)
    lib().orc_exchange_p2g(C.byref(p), C.byref(c), x.shape[1], _ptr(x, C.c_double), _ptr(r, C.c_double),
                           _ptr(held, C.c_double), _ptr(Fc, C.c_double), _ptr(Ffl, C.c_double), float(weight),
                           _ptr(fs, C.c_int64))
    return fs


def substeps(Dt, dt_max):
    return int(lib().orc_substeps(float(Dt), float(dt_max)))


def sand_step(cfg, Dt, x, v, r, u, alpha_fx, gp=None, af=None):
    """One sand step (Alg. 2) of length Dt in ceil(Dt / cfg dt) sub-steps.
    Returns dict(x, v, alpha, mom, fs, N)."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    r, u = _f64(r), _f64(u)
    gp = None if gp is None else _f64(gp)
    af = None if af is None else _f64(af)
    G = nodes(cfg)
    alpha = np.ascontiguousarray(alpha_fx, np.int64).copy()
    mom = np.zeros((3, G), np.int64)
    fs = np.zeros((3, G), np.int64)
    p, c = params(cfg), coupling(cfg)
    N = lib().orc_sand_step(C.byref(p), C.byref(c), x.shape[1], float(Dt), _ptr(x, C.c_double),
                            _ptr(v, C.c_double), _ptr(r, C.c_double), _ptr(u, C.c_double), _ptr(gp, C.c_double),
                            _ptr(af, C.c_double), _ptr(alpha, C.c_int64), _ptr(mom, C.c_int64),
                            _ptr(fs, C.c_int64))
    return dict(x=x, v=v, alpha=alpha, mom=mom, fs=fs, N=int(N))


# ---- capillary (concentration-gradient) pair force, Sec. 5.4 ---------------

def gamma(cfg, sr):
    return float(lib().orc_gamma(C.byref(capillary(cfg)), float(sr)))


def moisture_ratio(held, alpha_f):
    """sr_i = held_i + alpha_f,i / (1 - alpha_f,i) per granule."""
    held, alpha_f = _f64(held), _f64(alpha_f)
    sr = np.zeros(held.shape[0])
    lib().orc_moisture_ratio(held.shape[0], _ptr(held, C.c_double), _ptr(alpha_f, C.c_double), _ptr(sr, C.c_double))
    return sr


def bridge(cfg, rb):
    """(V*, d_r) of a pair of mean radius rb."""
    V, dr = np.zeros(1), np.zeros(1)
    lib().orc_bridge(C.byref(capillary(cfg)), float(rb), _ptr(V, C.c_double), _ptr(dr, C.c_double))
    return float(V[0]), float(dr[0])


def bridge_energy(cfg, rb, s):
    return float(lib().orc_bridge_energy(C.byref(capillary(cfg)), float(rb), float(s)))


def fst(cfg, rb, s):
    return float(lib().orc_fst(C.byref(capillary(cfg)), float(rb), float(s)))


def capillary_pair(cfg, xi, xj, ri, rj, sri, srj):
    """Capillary force of j on i (3,)."""
    F = np.zeros(3)
    a, b = _f64(xi), _f64(xj)
    lib().orc_capillary_pair_force(C.byref(capillary(cfg)), _ptr(a, C.c_double), _ptr(b, C.c_double), float(ri),
                                   float(rj), float(sri), float(srj), _ptr(F, C.c_double))
    return F


def capillary_forces(cfg, x, r, sr):
    """Capillary force on each granule (3,n) from every bridged pair."""
    x, r, sr = _f64(x), _f64(r), _f64(sr)
    F = np.zeros((3, x.shape[1]))
    lib().orc_capillary_forces(C.byref(params(cfg)), C.byref(capillary(cfg)), x.shape[1], _ptr(x, C.c_double),
                               _ptr(r, C.c_double), _ptr(sr, C.c_double), _ptr(F, C.c_double))
    return F


# ---- differentiable form (unquantised transfers) and its reverse pass -------

def contact_vjp(cfg, x, v, r, gF):
    """(gx, gv, gmu) = (dL/dx, dL/dv, dL/dmu) for dL/dF_c = gF."""
    x, v, r, gF = _f64(x), _f64(v), _f64(r), _f64(gF)
    gx = np.zeros_like(x)
    gv = np.zeros_like(v)
    gmu = np.zeros(1)
    p = params(cfg)
    lib().orc_contact_vjp(C.byref(p), x.shape[1], _ptr(x, C.c_double), _ptr(v, C.c_double), _ptr(r, C.c_double),
                          _ptr(gF, C.c_double), _ptr(gx, C.c_double), _ptr(gv, C.c_double), _ptr(gmu, C.c_double))
    return gx, gv, float(gmu[0])


def drag_vjp(cfg, r, v, u_at, alpha_f, gF):
    """(gv, gu_at, galpha_f, gcd) for dL/dF_d = gF."""
    r, v, u_at, alpha_f, gF = _f64(r), _f64(v), _f64(u_at), _f64(alpha_f), _f64(gF)
    gv = np.zeros_like(v)
    guat = np.zeros_like(u_at)
    gaf = np.zeros_like(alpha_f)
    gcd = np.zeros(1)
    p = params(cfg)
    lib().orc_drag_vjp(C.byref(p), r.shape[0], _ptr(r, C.c_double), _ptr(v, C.c_double), _ptr(u_at, C.c_double),
                       _ptr(alpha_f, C.c_double), _ptr(gF, C.c_double), _ptr(gv, C.c_double),
                       _ptr(guat, C.c_double), _ptr(gaf, C.c_double), _ptr(gcd, C.c_double))
    return gv, guat, gaf, float(gcd[0])


def g2p_vjp(cfg, x, u, alpha_real, guat, gaf):
    """(gx, galpha) for cotangents of u_at and alpha_f."""
    x, u, alpha_real, guat, gaf = _f64(x), _f64(u), _f64(alpha_real), _f64(guat), _f64(gaf)
    gx = np.zeros_like(x)
    galpha = np.zeros(nodes(cfg))
    p = params(cfg)
    lib().orc_g2p_vjp(C.byref(p), x.shape[1], _ptr(x, C.c_double), _ptr(u, C.c_double), _ptr(alpha_real, C.c_double),
                      _ptr(guat, C.c_double), _ptr(gaf, C.c_double), _ptr(gx, C.c_double), _ptr(galpha, C.c_double))
    return gx, galpha


def p2g_vjp(cfg, x, v, r, galpha=None, gmom=None):
    """(gx, gv) for cotangents of the real alpha grid and momentum grid."""
    x, v, r = _f64(x), _f64(v), _f64(r)
    ga = None if galpha is None else _f64(galpha)
    gm = None if gmom is None else _f64(gmom)
    gx = np.zeros_like(x)
    gv = np.zeros_like(v)
    p = params(cfg)
    lib().orc_p2g_vjp(C.byref(p), x.shape[1], _ptr(x, C.c_double), _ptr(v, C.c_double), _ptr(r, C.c_double),
                      _ptr(ga, C.c_double), _ptr(gm, C.c_double), _ptr(gx, C.c_double), _ptr(gv, C.c_double))
    return gx, gv


def rollout(cfg, x0, v0, r, u, steps, want_mom=False):
    """Real-mode rollout.  Returns (L, signature[, mom])."""
    x0, v0, r, u = _f64(x0), _f64(v0), _f64(r), _f64(u)
    mom = np.zeros((3, nodes(cfg))) if want_mom else None
    sig = (C.c_uint64 * 1)()
    p = params(cfg)
    L = lib().orc_rollout(C.byref(p), x0.shape[1], _ptr(x0, C.c_double), _ptr(v0, C.c_double), _ptr(r, C.c_double),
                          _ptr(u, C.c_double), int(steps), _ptr(mom, C.c_double), sig)
    return (L, int(sig[0]), mom) if want_mom else (L, int(sig[0]))


def rollout_vjp(cfg, x0, v0, r, u, steps):
    """Reverse pass: (L, dL/dv0 (3,n), dL/dmu, dL/dC_d)."""
    x0, v0, r, u = _f64(x0), _f64(v0), _f64(r), _f64(u)
    gv0 = np.zeros_like(v0)
    gmu = np.zeros(1)
    gcd = np.zeros(1)
    p = params(cfg)
    L = lib().orc_rollout_vjp(C.byref(p), x0.shape[1], _ptr(x0, C.c_double), _ptr(v0, C.c_double),
                              _ptr(r, C.c_double), _ptr(u, C.c_double), int(steps), _ptr(gv0, C.c_double),
                              _ptr(gmu, C.c_double), _ptr(gcd, C.c_double))
    return L, gv0, float(gmu[0]), float(gcd[0])
def capillary_forces_sample(cfg, x, r, sr, idx):
    """Capillary force (3, m) on the sampled granules idx and the sum of the
    magnitudes of their bridge forces (m,)."""
    x, r, sr = _f64(x), _f64(r), _f64(sr)
    idx = np.ascontiguousarray(idx, np.int64)
    m = idx.shape[0]
    F = np.zeros((3, m))
    fa = np.zeros(m)
    lib().orc_capillary_forces_sample(C.byref(params(cfg)), C.byref(capillary(cfg)), x.shape[1], _ptr(x, C.c_double),
                                      _ptr(r, C.c_double), _ptr(sr, C.c_double), m, _ptr(idx, C.c_int64),
                                      _ptr(F, C.c_double), _ptr(fa, C.c_double))
    return F, fa


# ---- wet granules (Sec. 5.3, Eq. 19) ----

def wet_mass(cfg, r, held):
    """m = V (rho_s + held rho_f) per granule."""
    r, held = _f64(r), _f64(held)
    m = np.zeros(r.shape[0])
    lib().orc_wet_mass(C.byref(params(cfg)), float(cfg.get("rho_f", 0.0)), r.shape[0], _ptr(r, C.c_double),
                       _ptr(held, C.c_double), _ptr(m, C.c_double))
    return m


def contact_forces_wet(cfg, x, v, r, m):
    """Contact forces with per-granule masses: (F (3,n), fabs (n), ncontacts (n))."""
    x, v, r, m = _f64(x), _f64(v), _f64(r), _f64(m)
    n = x.shape[1]
    F = np.zeros((3, n))
    fa = np.zeros(n)
    nc = np.zeros(n, np.int32)
    lib().orc_contact_forces_wet(C.byref(params(cfg)), n, _ptr(x, C.c_double), _ptr(v, C.c_double),
                                 _ptr(r, C.c_double), _ptr(m, C.c_double), _ptr(F, C.c_double),
                                 _ptr(fa, C.c_double), _ptr(nc, C.c_int32))
    return F, fa, nc


def contact_forces_sample_wet(cfg, x, v, r, m, idx):
    x, v, r, m = _f64(x), _f64(v), _f64(r), _f64(m)
    idx = np.ascontiguousarray(idx, np.int64)
    k = idx.shape[0]
    F = np.zeros((3, k))
    fa = np.zeros(k)
    lib().orc_contact_forces_sample_wet(C.byref(params(cfg)), x.shape[1], _ptr(x, C.c_double), _ptr(v, C.c_double),
                                        _ptr(r, C.c_double), _ptr(m, C.c_double), k, _ptr(idx, C.c_int64),
                                        _ptr(F, C.c_double), _ptr(fa, C.c_double))
    return F, fa


def integrate_wet(cfg, r, m, Fc, Fd, x, v, held=None):
    """(x, v) advanced with per-granule masses (virtual mass per cfg, with the
    volume V (1 + held) when held is given, Sec. 5.3)."""
    r, m, Fc, Fd = _f64(r), _f64(m), _f64(Fc), _f64(Fd)
    held = None if held is None else _f64(held)
    x, v = np.array(x, np.float64, order="C", copy=True), np.array(v, np.float64, order="C", copy=True)
    lib().orc_integrate_wet(C.byref(params(cfg)), C.byref(coupling(cfg)), r.shape[0], _ptr(r, C.c_double),
                            _ptr(held, C.c_double), _ptr(m, C.c_double), _ptr(Fc, C.c_double), _ptr(Fd, C.c_double),
                            _ptr(x, C.c_double), _ptr(v, C.c_double))
    return x, v


def p2g_fixed_wet(cfg, x, v, r, held):
    """(alpha (G,), mom (3, G)) of wet granules (Sec. 5.3): the fraction
    channel counts the held water's volume, frac (1 + held), and the momentum
    channels the wet mass."""
    x, v, r, held = _f64(x), _f64(v), _f64(r), _f64(held)
    G = nodes(cfg)
    a = np.zeros(G, np.int64)
    mo = np.zeros(3 * G, np.int64)
    lib().orc_p2g_fixed_wet(C.byref(params(cfg)), float(cfg.get("rho_f", 0.0)), x.shape[1], _ptr(x, C.c_double),
                            _ptr(v, C.c_double), _ptr(r, C.c_double), _ptr(held, C.c_double), _ptr(a, C.c_int64),
                            _ptr(mo, C.c_int64))
    return a, mo.reshape(3, G)


from . import idp  # noqa: E402,F401  (density projection, numpy/scipy)
