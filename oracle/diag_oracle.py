"""CPU reference of the experiment diagnostics of Sec. 4 (test
infrastructure: only tests/ use it; the product path never does).

Fields are numpy arrays of shape (nz, ny, nx) in 3-D and (1, ny, nx) or
(ny, nx) in 2-D and axisymmetric geometry (axis 0 of the problem = x or z along the last array
axis, axis 1 = y or r along the first), as the library stores them; a face
velocity array holds at index i the low face of cell i.  Positions are
cell-centre coordinates (cell i spans [i, i+1]).

- Falling drop (Sec. 4): U_drop = integral over phi > 0 of r u dr dz divided
  by the integral of r dr dz; the same mean without the weight r gives the
  3-D coalescence's W_drop.  u is taken at the cell centre as the mean of
  the cell's two faces (a boundary face beyond the last cell carries the
  boundary's value: 0 on walls and symmetry planes, the first face on a
  periodic axis).
- Interface positions (drop radius and half length, aspect ratio, fronts):
  phi = 0 crossings between neighbouring cell centres by linear
  interpolation.
"""
from __future__ import annotations

import math

import numpy as np


def _as3(a, dim):
    a = np.asarray(a, dtype=np.float64)
    return a if a.ndim == 3 else a.reshape((1,) + a.shape)  # 2-D (ny, nx) -> (1, ny, nx)


def _axis_of(dim, a):
    """numpy axis (of the 3-D view) of problem axis a"""
    if dim == 3:
        return 2 - a
    return {0: 2, 1: 1}[a]


def _centre(u, npaxis, periodic):
    """cell-centre mean of a face array along numpy axis npaxis"""
    hi = np.roll(u, -1, axis=npaxis)
    if not periodic:
        idx = [slice(None)] * u.ndim
        idx[npaxis] = -1
        hi[tuple(idx)] = 0.0
    return 0.5 * (u + hi)


def phase_stats(prob, state):
    """(volume, centroid[3], velocity[3]) of the region phi > 0."""
    dim = prob["dim"]
    axi = bool(prob.get("axisym", 0))
    phi = _as3(state["phi"], dim)
    nz, ny, nx = phi.shape
    zc, yc, xc = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    mask = phi > 0
    w = np.where(mask, yc if axi else 1.0, 0.0)  # axisymmetric: r is the first stored axis (y)
    vol = float(w.sum())
    comps = ("u", "v", "w")[:dim]
    cent, vel = [math.nan] * 3, [math.nan] * 3
    if vol > 0:
        coords = {0: xc, 1: yc, 2: zc} if dim == 3 else {0: xc, 1: yc}
        for a in range(dim):
            cent[a] = float((w * coords[a]).sum() / vol)
            npax = _axis_of(dim, a)
            bc_lo = prob["bc"][2 * a]
            uc = _centre(_as3(state[comps[a]], dim), npax, bc_lo == 0)
            vel[a] = float((w * uc).sum() / vol)
    return vol, cent, vel


def _crossings_1d(line):
    """positions of the sign changes (phi > 0 on exactly one side) along a line"""
    out = []
    for i in range(len(line) - 1):
        f0, f1 = float(line[i]), float(line[i + 1])
        if (f0 > 0) != (f1 > 0):
            out.append(i + 0.5 + f0 / (f0 - f1))
    return out


def line_crossings(prob, state, axis, i0, i1=0):
    """(first, last) crossing on the grid line along `axis` through the
    indices (i0, i1) of the other axes in increasing order."""
    dim = prob["dim"]
    phi = _as3(state["phi"], dim)
    others = [a for a in range(dim) if a != axis]
    idx = [slice(None)] * 3
    for a, v in zip(others, (i0, i1)):
        idx[_axis_of(dim, a)] = v
    if dim == 2:
        idx[0] = 0
    c = _crossings_1d(phi[tuple(idx)])
    return (min(c), max(c)) if c else (math.nan, math.nan)


def interface_extent(prob, state):
    """[(smallest, largest) crossing] along each axis over all grid lines."""
    dim = prob["dim"]
    phi = _as3(state["phi"], dim)
    out = []
    for a in range(3):
        if a >= dim:
            out.append((math.nan, math.nan))
            continue
        lines = np.moveaxis(phi, _axis_of(dim, a), -1).reshape(-1, phi.shape[_axis_of(dim, a)])
        c = [x for line in lines for x in _crossings_1d(line)]
        out.append((min(c), max(c)) if c else (math.nan, math.nan))
    return out
