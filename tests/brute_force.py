"""Brute-force global solve of the transport step on tiny meshes (numpy).

Independent of the oracle's sweep: the cell operator is taken from the
oracle's single-cell residual as a black box (L = responses to unit nodal
values, lift = responses to unit neighbour traces; that residual is pinned
separately against exact polynomial derivatives), and the whole implicit
system of one Jacobi iterate (Sec. 5.1, eq:ibvp) is assembled over ALL cells
and solved with numpy.linalg.solve, with no ordering at all.
"""
from __future__ import annotations

import itertools

import numpy as np


def cell_operator(orc, cfg, V):
    nn, d = cfg.nn, cfg.dim
    L = np.zeros((nn, nn))
    lift = np.zeros((2 * d, nn))
    zero_tr = np.zeros(2 * d * nn)
    for j in range(nn):
        e = np.zeros(nn)
        e[j] = 1.0
        L[:, j] = orc.cell_residual(cfg, V, e, zero_tr)
    for fce in range(2 * d):
        for i in range(nn):
            tr = np.zeros((2 * d, nn))
            tr[fce, i] = 1.0
            r = orc.cell_residual(cfg, V, np.zeros(nn), tr.ravel())
            lift[fce, i] = r[i]
            assert np.count_nonzero(np.abs(r) > 0) <= 1
    return L, lift


def _cells(N, d):
    for t in itertools.product(*[range(N[a]) for a in reversed(range(d))]):
        yield tuple(reversed(t))


def _cell_id(cc, N):
    i, mul = 0, 1
    for a, c in enumerate(cc):
        i += c * mul
        mul *= N[a]
    return i


def _node_idx(i, d, P):
    out = []
    for _ in range(d):
        out.append(i % P)
        i //= P
    return out


def _node_id(ii, P):
    j, mul = 0, 1
    for v in ii:
        j += v * mul
        mul *= P
    return j


def _boundary_index(spec, per, ax, side, cc, ii):
    """Boundary-node number of node ii of cell cc on face (ax, side): the faces
    of the non-periodic axes in x, y, z order, low end then high end; on a
    face, cells over the other axes then the cell's face nodes over the other
    axes' node indices (lower axis fastest)."""
    d = spec["dim"]
    N = spec["n_cells"][:d]
    P = spec["degree"] + 1
    def nodes_on(a):
        n = 1
        for o in range(d):
            if o != a:
                n *= N[o] * P
        return n
    off = sum(2 * nodes_on(a) for a in range(ax) if not per[a]) + side * nodes_on(ax)
    cell, cmul, node, nmul = 0, 1, 0, 1
    for o in range(d):
        if o == ax:
            continue
        cell += cc[o] * cmul
        cmul *= N[o]
        node += ii[o] * nmul
        nmul *= P
    return off + cell * nmul + node


def global_transport(orc, cfg, k, f_old, K, lagged=True, fb_old=None, fb_new=None):
    """K Jacobi iterates of the subdomain algorithm by dense global solves.

    lagged=False treats every face (wrap included) as implicit, i.e. the fully
    implicit periodic DG system (the limit K -> infinity).  On axes with
    spec["periodic"][a] == 0 the faces of the box take the prescribed inflow
    fb_old / fb_new (boundary-node numbering of _boundary_index).
    """
    spec = cfg.spec
    d, P, nn = cfg.dim, cfg.P, cfg.nn
    N = spec["n_cells"][:d]
    S = spec["sub_cells"][:d]
    dt, th = spec["dt"], spec.get("theta", 0.5)
    V = np.asarray(spec["vel"][k * d:(k + 1) * d], dtype=np.float64)
    L, lift = cell_operator(orc, cfg, V)
    ncell = cfg.ncell
    n = ncell * nn
    f_old = np.asarray(f_old, dtype=np.float64).reshape(n)
    per = list(spec.get("periodic", [1, 1, 1]))[:d]
    # face structure: (cell, face, neighbour cell or -1 at a Dirichlet face,
    # interface?, cell coordinates)
    faces = []
    for cc in _cells(N, d):
        cid = _cell_id(cc, N)
        for ax in range(d):
            for side in (0, 1):
                nc = list(cc)
                nc[ax] += 1 if side else -1
                wrapped = nc[ax] < 0 or nc[ax] >= N[ax]
                nc[ax] %= N[ax]
                iface = wrapped or (cc[ax] // S[ax] != nc[ax] // S[ax])
                nb = -1 if (wrapped and not per[ax]) else _cell_id(nc, N)
                faces.append((cid, 2 * ax + side, nb, iface, cc))
    prev = f_old.copy()
    iters = K if lagged else 1
    for _ in range(iters):
        A = np.zeros((n, n))
        b = np.zeros(n)
        for cid in range(ncell):
            sl = slice(cid * nn, (cid + 1) * nn)
            A[sl, sl] += np.eye(nn) / dt + th * L
            b[sl] += f_old[sl] / dt - (1 - th) * (L @ f_old[sl])
        for cid, fce, nb, iface, cc in faces:
            ax, side = divmod(fce, 2)
            for i in range(nn):
                c = lift[fce, i]
                if c == 0.0:
                    continue
                ii = _node_idx(i, d, P)
                if nb < 0:
                    bi = _boundary_index(spec, per, ax, side, cc, ii)
                    bo = 0.0 if fb_old is None else fb_old[bi]
                    bn = 0.0 if fb_new is None else fb_new[bi]
                    b[cid * nn + i] -= c * ((1 - th) * bo + th * bn)
                    continue
                ii[ax] = 0 if side else P - 1
                j = _node_id(ii, P)
                row = cid * nn + i
                col = nb * nn + j
                b[row] -= (1 - th) * c * f_old[col]
                if lagged and iface:
                    b[row] -= th * c * prev[col]
                else:
                    A[row, col] += th * c
        prev = np.linalg.solve(A, b)
    return prev.reshape(ncell, nn)
