"""FP64 CPU oracle of the density projection (IDP) of the fluid fraction --
TEST INFRASTRUCTURE, like the rest of this package.

Sec. 5.1: the sand fraction alpha_s at cell centres (Eq. 7a, the P2G grid,
clamped at 0.740) fixes the target fluid fraction alpha_f' = 1 - alpha_s; the
fluid particles' own fraction alpha_f* (Eq. 7b) is an input.  Eq. 12b,

    (dt^2 / (alpha_f' rho_0)) div(alpha_f' grad p_2) = 1 - alpha_f* / alpha_f',

is discretised on the MAC grid as in App. B: cell-centred pressure, face
coefficients beta = (alpha_f'(c) + alpha_f'(j)) / 2, so that with the scaled
pressure q = (dt^2 / (rho_0 dx^2)) p_2 every fluid cell c satisfies

    (L q)_c = sum_j beta_cj (q_c - q_j) = alpha_f'(c) (clamp(alpha_f*/alpha_f', 0.5, 1.5) - 1)

(the sign of Eq. 12b; App. B prints the same operator with the opposite sign
on its right-hand side, a reading recorded in the design notes).  Neighbours
j are the six face neighbours; an air cell is a Dirichlet neighbour (p = 0,
its beta uses its own alpha_f'), a solid cell or the box boundary closes the
face (Neumann, no term).  The position change on a face (Eq. 13) is
dx_face = -(dt^2 / rho_0) grad p_2 = -dx (q_j - q_c) along the face normal,
clamped to one cell width (Sec. 5.1).

Cell labels: 0 fluid, 1 air, 2 solid.  Grids are numpy arrays of shape
(nz, ny, nx) (x fastest in memory, as on the device).
"""
import numpy as np

FLUID, AIR, SOLID = 0, 1, 2


def target_fraction(alpha_fx, alpha_max, absorb_max=0.0):
    """alpha_f' = 1 - min(alpha * 2^-32, alpha_max (1 + absorb_max)) from the
    int64 P2G grid (Eq. 7a in 2^-32 cell volumes; the densest-packing clamp
    of Sec. 5.1, raised by the maximum absorption ratio of Sec. 5.3 when the
    granules hold water: the water fills part of the voids)."""
    amax = alpha_max * (1.0 + absorb_max)
    a_s = np.minimum(np.asarray(alpha_fx, np.int64).astype(np.float64) * 2.0 ** -32, amax)
    return 1.0 - a_s


def rhs(alpha_t, alpha_star, label):
    """Right-hand side of the scaled Eq. 12b per cell: alpha_f' (ratio - 1)
    with ratio = alpha_f* / alpha_f' clamped to [0.5, 1.5]; zero off fluid."""
    ratio = np.clip(np.asarray(alpha_star, np.float64) / alpha_t, 0.5, 1.5)
    return np.where(label == FLUID, alpha_t * (ratio - 1.0), 0.0)


def _shift(a, axis, step, fill):
    """b[c] = a[c + step e_axis], `fill` outside the box."""
    b = np.full_like(a, fill)
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    if step > 0:
        src[axis], dst[axis] = slice(step, None), slice(None, -step)
    else:
        src[axis], dst[axis] = slice(None, step), slice(-step, None)
    b[tuple(dst)] = a[tuple(src)]
    return b


# neighbour order of the per-cell sums: -x, +x, -y, +y, -z, +z (array axes 2, 1, 0)
_NEIGHBOURS = [(2, -1), (2, 1), (1, -1), (1, 1), (0, -1), (0, 1)]


def _faces(alpha_t, label):
    """Per neighbour: (open face mask, beta, neighbour label) for every cell."""
    out = []
    for axis, step in _NEIGHBOURS:
        lj = _shift(label, axis, step, SOLID)
        aj = _shift(alpha_t, axis, step, 0.0)
        open_ = (label == FLUID) & (lj != SOLID)
        beta = (alpha_t + aj) * 0.5
        out.append((axis, step, open_, beta, lj))
    return out


def apply(alpha_t, label, q):
    """(L q) on fluid cells, summed over the neighbours in the fixed order;
    q on other cells is taken as its own row (identity), so L is SPD on the
    whole grid and a solution is zero off the fluid."""
    qf = np.where(label == FLUID, q, 0.0)
    acc = np.zeros_like(alpha_t)
    for axis, step, open_, beta, lj in _faces(alpha_t, label):
        qj = _shift(qf, axis, step, 0.0)
        acc = acc + np.where(open_, beta * (qf - qj), 0.0)
    return np.where(label == FLUID, acc, q)


def diagonal(alpha_t, label):
    """Diagonal of L: sum of the open faces' beta on fluid cells, 1 elsewhere."""
    acc = np.zeros_like(alpha_t)
    for axis, step, open_, beta, lj in _faces(alpha_t, label):
        acc = acc + np.where(open_, beta, 0.0)
    return np.where(label == FLUID, acc, 1.0)


def matrix(alpha_t, label):
    """L assembled as a sparse matrix over all cells (row per cell, x fastest),
    entry by entry from the face list: the diagonal takes beta of every open
    face, the off-diagonal -beta of every face to a fluid neighbour."""
    import scipy.sparse as sp
    nz, ny, nx = label.shape
    N = label.size
    idx = np.arange(N).reshape(label.shape)
    rows, cols, vals = [], [], []
    fl = label == FLUID
    diag = np.where(fl, 0.0, 1.0)
    for axis, step, open_, beta, lj in _faces(alpha_t, label):
        diag = diag + np.where(open_, beta, 0.0)
        both = open_ & (lj == FLUID)
        j = _shift(idx, axis, step, -1)
        rows.append(idx[both])
        cols.append(j[both])
        vals.append(-beta[both])
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def solve(alpha_t, label, s):
    """Direct sparse solution of L q = s (fluid rows; zero elsewhere)."""
    import scipy.sparse.linalg as spl
    A = matrix(alpha_t, label).tocsc()
    b = np.where(label == FLUID, s, 0.0).ravel()
    return spl.spsolve(A, b).reshape(label.shape)


def displacement(q, label, dx):
    """Position change on the MAC faces, Eq. 13 in the scaled pressure:
    d = dx (q_c - q_j) for the face from cell c to its +axis neighbour j (a
    positive d moves fluid along +axis), where at least one side is fluid
    and neither is solid (air sides count as q = 0); clamped to [-dx, dx].
    Returns the x-, y- and z-face arrays of shapes (nz, ny, nx + 1),
    (nz, ny + 1, nx), (nz + 1, ny, nx); faces on the box boundary are zero."""
    qf = np.where(label == FLUID, q, 0.0)
    out = []
    for axis in (2, 1, 0):
        lj = _shift(label, axis, 1, SOLID)
        qj = _shift(qf, axis, 1, 0.0)
        live = ((label == FLUID) | (lj == FLUID)) & (label != SOLID) & (lj != SOLID)
        d = np.where(live, np.clip(dx * (qf - qj), -dx, dx), 0.0)
        shape = list(label.shape)
        shape[axis] += 1
        f = np.zeros(shape)
        sl = [slice(None)] * 3
        sl[axis] = slice(1, label.shape[axis] + 1)
        f[tuple(sl)] = d  # face i + 1/2 stored at index i + 1
        out.append(f)
    return tuple(out)


def projection(alpha_fx, alpha_max, alpha_star, label, dx, absorb_max=0.0):
    """The whole density projection: target fraction, right-hand side,
    direct solve and face displacements.  Returns (alpha_t, s, q, faces)."""
    alpha_t = target_fraction(alpha_fx, alpha_max, absorb_max)
    s = rhs(alpha_t, alpha_star, label)
    q = solve(alpha_t, label, s)
    return alpha_t, s, q, displacement(q, label, dx)
