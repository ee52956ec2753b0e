"""Error norms of the parity tests (GPU result against the FP64 oracle).

relerr: max |a - b| / max |b| over every node, component (and velocity):
the norm the tolerances 1e-12 (FP64) / 1e-5 (FP32) are stated in.

relerr_planes: the same per (velocity, component) plane of F, or per
component of W, each divided by that plane's own max |b|; the largest over
the planes.  A component much smaller than the others (Euler momentum ~0.1
beside energy ~2.5) is then held to the tolerance on its own scale.  A plane
whose reference is below `floor` times the global max |b| has no scale of its
own (it is zero in exact arithmetic, e.g. the kinetic function of the
velocity that sits exactly on the sub-characteristic bound, whose equilibrium
vanishes: its values are rounding noise) and is measured on the global scale.

Layouts: W [cell][node][c], F [k][cell][node][c] (the C ABI's).

outflow_nodes: the values of one velocity's field at the nodes on the
subdomains' outflow faces (where the subdomain iteration's traces live).
"""
from __future__ import annotations

import numpy as np


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def relerr_planes(a, b, floor=1e-6):
    a = np.asarray(a)
    b = np.asarray(b)
    if a.ndim == 4:
        red = (1, 2)
    elif a.ndim == 3:
        red = (0, 1)
    else:
        raise ValueError("expected W [cell][node][c] or F [k][cell][node][c]")
    gmax = float(np.max(np.abs(b)))
    num = np.max(np.abs(a - b), axis=red)
    pmax = np.max(np.abs(b), axis=red)
    den = np.where(pmax >= floor * gmax, pmax, gmax)
    return float(np.max(num / den))


def errors(W, Wref, F, Fref):
    """(global W, global F, per-plane W, per-plane F) relative errors."""
    return (relerr(W, Wref), relerr(F, Fref), relerr_planes(W, Wref), relerr_planes(F, Fref))


def check(W, Wref, F, Fref, tol, label="", tol_plane=None):
    """Global errors <= tol, per-plane errors <= tol_plane (default tol)."""
    tol_plane = tol if tol_plane is None else tol_plane
    ew, ef, pw, pf = errors(W, Wref, F, Fref)
    print("  %s rel err W %.3e F %.3e | per plane W %.3e F %.3e" % (label, ew, ef, pw, pf),
          flush=True)
    assert max(ew, ef) <= tol and max(pw, pf) <= tol_plane, (ew, ef, pw, pf)
    return ew, ef, pw, pf


def outflow_nodes(c, k, T):
    """T[cell, node] of velocity k -> its values at the nodes on the
    subdomains' outflow faces: for each axis a with V^a != 0, the nodes at
    the downwind end along a of the cells at the downwind end of their
    subdomain along a."""
    spec = c.spec
    d, P = c.dim, c.P
    v = np.asarray(spec["vel"], dtype=np.float64).reshape(-1, d)[k]
    N = [int(n) for n in spec["n_cells"][:d]]
    S = [int(x) for x in spec["sub_cells"][:d]]
    # cells and nodes numbered with axis 0 fastest
    cc = np.indices(N[::-1]).reshape(d, -1)[::-1]        # [axis][cell]
    nc = np.indices([P] * d).reshape(d, -1)[::-1]        # [axis][node]
    mask = np.zeros((len(cc[0]), len(nc[0])), dtype=bool)
    for a in range(d):
        if v[a] > 0:
            mask |= ((cc[a] % S[a]) == S[a] - 1)[:, None] & (nc[a] == P - 1)[None, :]
        elif v[a] < 0:
            mask |= ((cc[a] % S[a]) == 0)[:, None] & (nc[a] == 0)[None, :]
    return T[mask]
