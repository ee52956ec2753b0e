"""Seeded synthetic workloads (problem descriptions and initial states).

This module holds no arithmetic of the kinetic scheme: it only describes the
problems (grid, degree, law, kinetic velocities, omega, dt) and samples the
initial conserved state W0 at the interpolation points.  Both the GPU path and
the CPU oracle take their inputs from here; neither is imported by it.

The meshes, experiments and data sets of the paper are not available; these
seeded Cartesian problems stand in for them (periodic unit boxes).

* ``time step``: dt = beta * h_min / lambda_max with h_min = volume/surface of
  a cell (h / (2 d) on a cube) and lambda_max the largest wave speed of the
  conservation law (definition of the CFL number in Sec. 6.1.2, eq:def_CFL).
* ``kinetic velocities``: +-lambda e_i (D2Q4 / D3Q6); lambda is chosen above the
  largest wave speed (sub-characteristic condition, Sec. 2.1), on the bound
  lambda >= d * max spectral radius for acoustics and advection, and 1.1 times
  that bound for Euler.

Node coordinates for sampling are computed here with numpy's Legendre module
(Gauss-Lobatto points = end points + roots of P_p'); they are input sampling
positions only.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 2212110100

LAW_LINEAR = 0
LAW_EULER = 1


def gl_points(p: int) -> np.ndarray:
    """Gauss-Lobatto points on [0, 1] (p + 1 points); p = 0 -> midpoint."""
    if p == 0:
        return np.array([0.5])
    leg = np.polynomial.legendre.Legendre.basis(p).deriv()
    inner = np.sort(np.real(leg.roots())) if p > 1 else np.array([])
    x = np.concatenate(([-1.0], inner, [1.0]))
    return 0.5 * (x + 1.0)


def node_coords(spec: dict) -> np.ndarray:
    """Physical coordinates, shape [n_cell, n_node, dim], cells and nodes x-fastest."""
    d = spec["dim"]
    N = spec["n_cells"][:d]
    lo = np.asarray(spec["box_lo"][:d], dtype=np.float64)
    hi = np.asarray(spec["box_hi"][:d], dtype=np.float64)
    h = (hi - lo) / np.asarray(N)
    xi = gl_points(spec["degree"])
    P = len(xi)
    # cell coordinate grids (x fastest) and node offsets (x fastest)
    cidx = np.indices(tuple(reversed(N))).reshape(d, -1)[::-1]  # [d, ncell]
    nidx = np.indices((P,) * d).reshape(d, -1)[::-1]              # [d, nn]
    X = np.empty((cidx.shape[1], nidx.shape[1], d))
    for a in range(d):
        X[:, :, a] = lo[a] + h[a] * (cidx[a][:, None] + xi[nidx[a]][None, :])
    return X


def d2q4(lam: float) -> list[float]:
    return [lam, 0.0, -lam, 0.0, 0.0, lam, 0.0, -lam]


def d3q6(lam: float) -> list[float]:
    v = []
    for a in range(3):
        for s in (1.0, -1.0):
            e = [0.0, 0.0, 0.0]
            e[a] = s * lam
            v += e
    return v


def d3q4(lam: float) -> list[float]:
    """The paper's D3Q4 set (Sec. 6.1.3): lambda (1,1,1), (1,-1,-1), (-1,1,-1), (-1,-1,1)."""
    return [lam, lam, lam, lam, -lam, -lam, -lam, lam, -lam, -lam, -lam, lam]


def maxwell_params() -> list[float]:
    """Q^i = A^i W for W = (E, H), Q(W, N) = (-N x H, N x E) (Sec. 6.1.1)."""
    A = np.zeros((3, 6, 6))
    for i in range(3):
        e = np.zeros(3)
        e[i] = 1.0
        for col in range(3):
            u = np.zeros(3)
            u[col] = 1.0
            A[i, 0:3, 3 + col] = -np.cross(e, u)
            A[i, 3:6, col] = np.cross(e, u)
    return [float(v) for v in A.ravel()]


def w_plane_wave(X, t, freq=1):
    """Plane wave of Sec. 6.2: E_z = cos(2 pi nu (x - t)), H_y = -E_z."""
    W = np.zeros(X.shape[:-1] + (6,))
    c = np.cos(2 * np.pi * freq * (X[..., 0] - t))
    W[..., 2] = c
    W[..., 4] = -c
    return W


def _box(d):
    return [0.0] * 3, [1.0 if a < d else 1.0 for a in range(3)]


def _pad3(x, fill=1):
    x = list(x)
    return x + [fill] * (3 - len(x))


def _dt(beta, h, d, lam_max):
    return beta * (h / (2.0 * d)) / lam_max


# --------------------------------------------------------------------------
# initial states (recipes stated in the design doc)
# --------------------------------------------------------------------------

def _min_image(dx):
    return dx - np.round(dx)


def w0_advection(X, rng):
    """Gaussian pulse at (1/2, 1/2), width 0.08, plus 8 Fourier modes."""
    r2 = np.sum(_min_image(X - 0.5) ** 2, axis=-1)
    w = np.exp(-r2 / (2 * 0.08 ** 2))
    for _ in range(8):
        A = rng.uniform(-0.1, 0.1)
        while True:
            k = rng.integers(-4, 5, size=X.shape[-1])
            if np.any(k != 0):
                break
        phi = rng.uniform(0, 2 * np.pi)
        w = w + A * np.sin(2 * np.pi * (X @ k) + phi)
    return w[..., None]


def w0_acoustics(X, rng):
    """Sum of 16 Gaussian pressure pulses; zero velocity."""
    d = X.shape[-1]
    pr = np.zeros(X.shape[:-1])
    for _ in range(16):
        a = rng.uniform(0.5, 1.0)
        c = rng.uniform(0.0, 1.0, size=d)
        s = rng.uniform(0.01, 0.03)
        r2 = np.sum(_min_image(X - c) ** 2, axis=-1)
        pr += a * np.exp(-r2 / (2 * s * s))
    W = np.zeros(X.shape[:-1] + (1 + d,))
    W[..., 0] = pr
    return W


def w0_euler(X, rng, gamma=1.4):
    """rho = 1 + 0.2 s/max|s|, p = 1, u = 0.1 v/max|v| with v divergence-free."""
    d = X.shape[-1]
    s = np.zeros(X.shape[:-1])
    v = np.zeros(X.shape[:-1] + (d,))
    for _ in range(8):
        while True:
            k = rng.integers(-3, 4, size=d)
            if np.any(k != 0):
                break
        phi = rng.uniform(0, 2 * np.pi)
        s += np.sin(2 * np.pi * (X @ k) + phi)
    for _ in range(8):
        while True:
            k = rng.integers(-3, 4, size=d)
            if np.any(k != 0):
                break
        phi = rng.uniform(0, 2 * np.pi)
        r = rng.normal(size=d)
        e = r - (r @ k) / (k @ k) * k        # component orthogonal to k
        e = e / np.linalg.norm(e)
        v += e * np.cos(2 * np.pi * (X @ k) + phi)[..., None]
    rho = 1.0 + 0.2 * s / np.max(np.abs(s))
    u = 0.1 * v / np.max(np.linalg.norm(v, axis=-1))
    pr = np.ones_like(rho)
    W = np.empty(X.shape[:-1] + (d + 2,))
    W[..., 0] = rho
    W[..., 1:1 + d] = rho[..., None] * u
    W[..., d + 1] = pr / (gamma - 1.0) + 0.5 * rho * np.sum(u * u, axis=-1)
    return W


def euler_speeds(W, d, gamma=1.4):
    """(max |u| + c, max_i |u_i| + c) over the sampled nodes."""
    rho = W[..., 0]
    u = W[..., 1:1 + d] / rho[..., None]
    pr = (gamma - 1.0) * (W[..., d + 1] - 0.5 * rho * np.sum(u * u, axis=-1))
    c = np.sqrt(gamma * pr / rho)
    return float(np.max(np.linalg.norm(u, axis=-1) + c)), float(np.max(np.abs(u).max(axis=-1) + c))


# --------------------------------------------------------------------------
# problem descriptions
# --------------------------------------------------------------------------

def make_workload(cfg: int, n_cells=None, sub_cells=None, degree=None, steps=None,
                  beta=None, omega=None, n_iter=3, theta=0.5, seed=None,
                  precision="fp32", source_sigma=None, speed_bound=False, periodic=None):
    """Return (spec, W0) for workload ``cfg`` (1..4, 6), optionally resized.

    6 is the paper's own setting: Maxwell's equations with the D3Q4 velocity
    set, a plane wave along x (Sec. 6.2) in the periodic unit cube.

    spec is a plain dict (problem description); W0 has shape [cell, node, m].
    speed_bound (Euler): take lambda and dt from the bounds |u| <= 0.1,
    c <= sqrt(gamma p / 0.8) that every state of the Euler recipe satisfies,
    instead of the sampled maxima (the spec then does not depend on W0).
    """
    seed = SEED_BASE + cfg if seed is None else seed
    rng = np.random.default_rng(seed)
    if cfg == 1:
        d, p, m = 2, 1, 1
        N = n_cells or [32, 32]
        S = sub_cells or list(N)
        beta = 4.0 if beta is None else beta
        omega = 1.9 if omega is None else omega
        steps = 20 if steps is None else steps
        a = (1.0, 0.5)
        params = [a[0], a[1]]          # A^x = [a_x], A^y = [a_y]  (m = 1)
        lam = 2.0
        lam_max = math.hypot(*a)
        law = LAW_LINEAR
        vel = d2q4(lam)
        name = "advection2d_q1"
    elif cfg == 2:
        d, p, m = 2, 2, 3
        N = n_cells or [256, 256]
        S = sub_cells or [32, 32]
        beta = 10.0 if beta is None else beta
        omega = 2.0 if omega is None else omega
        steps = 100 if steps is None else steps
        c = 1.0
        Ax = [[0, c, 0], [c, 0, 0], [0, 0, 0]]
        Ay = [[0, 0, c], [0, 0, 0], [c, 0, 0]]
        params = [float(v) for row in Ax + Ay for v in row]
        lam = 2.0 * c
        lam_max = c
        law = LAW_LINEAR
        vel = d2q4(lam)
        name = "acoustics2d_q2"
    elif cfg == 6:
        d, p, m = 3, 2, 6
        N = n_cells or [16, 16, 16]
        S = sub_cells or [4, 4, 4]
        beta = 8.0 if beta is None else beta
        omega = (2.0 - 1e-12) if omega is None else omega
        steps = 10 if steps is None else steps
        params = maxwell_params()
        lam = math.sqrt(3.0)
        lam_max = 1.0
        law = LAW_LINEAR
        vel = d3q4(lam)
        name = "maxwell3d_d3q4_q2"
    elif cfg in (3, 4):
        d, m = 3, 5
        p = 2 if cfg == 3 else 3
        N = n_cells or ([128] * 3 if cfg == 3 else [96] * 3)
        S = sub_cells or ([16] * 3 if cfg == 3 else [12] * 3)
        beta = (8.0 if cfg == 3 else 20.0) if beta is None else beta
        omega = 1.9 if omega is None else omega
        steps = 50 if steps is None else steps
        params = [1.4]
        law = LAW_EULER
        lam = None
        name = "euler3d"
    else:
        raise ValueError("unknown workload %r" % cfg)
    if degree is not None:
        p = degree
    if name in ("euler3d", "acoustics2d_q2") and degree is not None:
        name = name.split("_q")[0] + "_q%d" % p
    elif name == "euler3d":
        name = "euler3d_q%d" % p
    N = list(N)
    S = list(S)
    spec = {
        "name": name, "cfg": cfg, "dim": d, "n_cells": _pad3(N), "sub_cells": _pad3(S),
        "box_lo": [0.0, 0.0, 0.0], "box_hi": [1.0, 1.0, 1.0], "degree": p, "m": m,
        "law": law, "law_params": params, "omega": float(omega), "theta": float(theta),
        "n_iter": int(n_iter), "steps": int(steps), "beta": float(beta), "seed": seed,
        "precision": precision,
        "source_sigma": None if source_sigma is None else [float(v) for v in source_sigma],
        "periodic": [1, 1, 1] if periodic is None else [int(v) for v in _pad3(periodic)],
    }
    X = node_coords(spec)
    if cfg == 6:
        W0 = w_plane_wave(X, 0.0)
    elif cfg == 1:
        W0 = w0_advection(X, rng)
    elif cfg == 2:
        W0 = w0_acoustics(X, rng)
    else:
        W0 = w0_euler(X, rng)
        if speed_bound:
            lam_max = lam_axis = 0.1 + math.sqrt(1.4 / 0.8)
        else:
            lam_max, lam_axis = euler_speeds(W0, d)
        lam = 1.1 * d * lam_axis
        vel = d3q6(lam)
    h = 1.0 / N[0]
    spec["lam"] = float(lam)
    spec["lam_max"] = float(lam_max)
    spec["vel"] = [float(v) for v in vel]
    spec["n_vel"] = len(vel) // d
    spec["dt"] = float(_dt(beta, h, d, lam_max))
    spec["kinetic_courant"] = float(lam * spec["dt"] / h)
    return spec, np.ascontiguousarray(W0, dtype=np.float64)


def boundary_faces(spec: dict):
    """(axis, side, first boundary node, node count) of every face of the box
    on a non-periodic axis, in the boundary-node order: axes x, y, z, low end
    then high end."""
    d = spec["dim"]
    P = spec["degree"] + 1
    N = spec["n_cells"][:d]
    per = spec.get("periodic", [1, 1, 1])
    out, off = [], 0
    for a in range(d):
        if per[a]:
            continue
        n = 1
        for o in range(d):
            if o != a:
                n *= N[o] * P
        for side in (0, 1):
            out.append((a, side, off, n))
            off += n
    return out


def n_boundary_nodes(spec: dict) -> int:
    return sum(f[3] for f in boundary_faces(spec))


def boundary_cells_nodes(spec: dict):
    """For every boundary node: (cell index, node index inside the cell) of the
    grid node that sits on it (the boundary cell's node on that face; degree 0:
    the cell's single node).  Face order of boundary_faces; on a face, cells
    over the other axes, then the cell's face nodes over the other axes' node
    indices (lower axis fastest)."""
    d = spec["dim"]
    P = spec["degree"] + 1
    N = spec["n_cells"][:d]
    cells, nodes = [], []
    for a, side, _, _ in boundary_faces(spec):
        others = [o for o in range(d) if o != a]
        for fc in np.ndindex(*[N[o] for o in reversed(others)]):
            fc = list(reversed(fc))
            for fn in np.ndindex(*[P for _ in others]):
                fn = list(reversed(fn))
                cc = [0] * d
                ii = [0] * d
                cc[a] = 0 if side == 0 else N[a] - 1
                ii[a] = 0 if side == 0 else P - 1
                for j, o in enumerate(others):
                    cc[o] = fc[j]
                    ii[o] = fn[j]
                cid, mul = 0, 1
                for o in range(d):
                    cid += cc[o] * mul
                    mul *= N[o]
                nid, mul = 0, 1
                for o in range(d):
                    nid += ii[o] * mul
                    mul *= P
                cells.append(cid)
                nodes.append(nid)
    return np.asarray(cells, dtype=np.int64), np.asarray(nodes, dtype=np.int64)


def boundary_coords(spec: dict) -> np.ndarray:
    """Coordinates [boundary node, dim] of the boundary nodes."""
    cells, nodes = boundary_cells_nodes(spec)
    X = node_coords(spec)
    return X[cells, nodes]


def boundary_state(spec: dict, W0=None, t: float = 0.0) -> np.ndarray:
    """Dirichlet data W_b [boundary node, m]: the exact plane wave at time t
    for the Maxwell workload, else the trace of the initial state W0 on the
    boundary (held constant in time)."""
    if spec.get("cfg") == 6:
        return np.ascontiguousarray(w_plane_wave(boundary_coords(spec), t), dtype=np.float64)
    cells, nodes = boundary_cells_nodes(spec)
    return np.ascontiguousarray(W0[cells, nodes], dtype=np.float64)


def unknowns(spec: dict) -> int:
    """U = cells * nodes * m * n_vel (scalar kinetic unknowns per step)."""
    d = spec["dim"]
    ncell = int(np.prod(spec["n_cells"][:d]))
    return ncell * (spec["degree"] + 1) ** d * spec["m"] * spec["n_vel"]


# --------------------------------------------------------------------------
# many uneven problems advanced together (batched launches)
# --------------------------------------------------------------------------

BATCH_ACOUSTICS_N = (64, 128, 256, 512)
BATCH_EULER_N = (32, 48, 64, 96)


def _batch_sub(N, nu, rng):
    """A subdomain width S dividing N with nu <= S (the subdomain iteration
    condition of Sec. 5.1 with the kinetic speed), drawn among the divisors
    8 <= S <= N; the line schedule's cost hardly depends on S."""
    need = max(8, math.ceil(nu))
    cands = [s for s in range(need, N + 1) if N % s == 0]
    return int(rng.choice(cands))


def make_batch_workload(n_problems=48, max_unknowns=4.0e9, acoustics_n=BATCH_ACOUSTICS_N,
                        euler_n=BATCH_EULER_N, euler_fraction=1.0 / 3.0, seed=None,
                        steps=20):
    """A seeded list of problem specs of uneven sizes: 2-D acoustics of degree
    1..3 on N^2 grids and 3-D Euler of degree 1..2 on N^3 grids, N drawn from
    the given lists, subdomain widths drawn with nu <= S, the total number of
    kinetic unknowns kept below max_unknowns (a draw that does not fit is
    redrawn; after 50 failed draws the smallest size is used).  The specs do
    not depend on the initial states; batch_member_state(spec) samples W0."""
    seed = SEED_BASE + 5 if seed is None else seed
    rng = np.random.default_rng(seed)
    out = []
    total = 0
    for i in range(n_problems):
        euler = rng.random() < euler_fraction
        for _ in range(50):
            if euler:
                p = int(rng.integers(1, 3))
                N = int(rng.choice(euler_n))
                u = N ** 3 * (p + 1) ** 3 * 5 * 6
            else:
                p = int(rng.integers(1, 4))
                N = int(rng.choice(acoustics_n))
                u = N ** 2 * (p + 1) ** 2 * 3 * 4
            if total + u <= max_unknowns:
                break
        else:
            p = 1
            N = int(min(euler_n if euler else acoustics_n))
        d = 3 if euler else 2
        nu = (1.1 * d * 8.0 / (2 * d)) if euler else 5.0   # lambda dt / h of the recipe
        S = _batch_sub(N, nu, rng)
        args = {"cfg": 3 if euler else 2, "n_cells": [N] * d, "sub_cells": [S] * d,
                "degree": p, "steps": steps, "seed": seed * 1000 + i}
        spec = _member(args, with_state=False)
        spec["name"] = "batch%02d_%s_%d" % (i, spec["name"], N)
        spec["member_args"] = args
        total += unknowns(spec)
        out.append(spec)
    return out


def _member(args, with_state):
    a = dict(args)
    cfg = a.pop("cfg")
    if not with_state:
        # the spec of a member does not depend on its state: build it on a
        # one-cell grid of the same kind and substitute the sizes
        d = len(a["n_cells"])
        small = dict(a, n_cells=[1] * d, sub_cells=[1] * d)
        spec, _ = make_workload(cfg, speed_bound=(cfg == 3), **small)
        N = a["n_cells"][0]
        spec["n_cells"] = _pad3(a["n_cells"])
        spec["sub_cells"] = _pad3(a["sub_cells"])
        spec["dt"] = float(_dt(spec["beta"], 1.0 / N, d, spec["lam_max"]))
        spec["kinetic_courant"] = float(spec["lam"] * spec["dt"] * N)
        return spec
    spec, W0 = make_workload(cfg, speed_bound=(cfg == 3), **a)
    return (spec, W0) if with_state else spec


def batch_member_state(spec):
    """The seeded initial state W0 [cell, node, m] of a batch member."""
    return _member(spec["member_args"], with_state=True)[1]
