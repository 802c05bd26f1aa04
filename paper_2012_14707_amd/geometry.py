"""Seeded synthetic problem generators: solid masks and wall-link tables with exact distance ratios.

This module produces *inputs* only.  It holds none of the lattice-Boltzmann arithmetic: it
rasterises walls onto the D2Q9 lattice and measures, for every link from a fluid node to a
solid node, the distance ratio gamma = |x_b - x_f| / |x_r - x_f| of the paper's Fig. 1
(Sec. III.A), together with the wall velocity at the crossing point x_b.  Both the GPU library
and the reference oracle consume what it returns.

A problem is a dict:
  params : physical inputs (Kn, H, body acceleration, periodicity, ...); nothing derived
  solid  : uint8 [ny, nx], 1 = solid (a closed set: nodes on a wall are solid)
  links  : dict of equal-length arrays
           x, y  (int32)  fluid node x_f
           dir   (int32)  D2Q9 direction 1..8 pointing from x_f toward the solid node x_r
           q     (float64) gamma in (0, 1]
           ubx, uby (float64) wall velocity at x_b
  meta   : geometry facts for analytic comparisons (H, radii, centre, ...)

Directions follow the paper's Eq. (Eq3): 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE.
"""
import math

import numpy as np

# D2Q9 direction vectors in the paper's order (Eq. (Eq3)); geometry needs only the vectors.
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.int64)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.int64)


def base_params(**kw):
    """Physical inputs with the paper's non-hydrodynamic relaxation times (Sec. IV)."""
    p = dict(periodic_x=0, periodic_y=0, kn=0.0, h=1.0, sigma=1.0, L1=math.nan, L2=math.nan, E=math.nan,
             tau_rho=1.0, tau_e=1.1, tau_eps=1.2, tau_j=1.0, tau_s_override=0.0, tau_q_override=0.0,
             r_override=0.0, l_override=0.0, l_mode="paper", r_mode="from_leff", diffuse="node",
             ax=0.0, ay=0.0, rho0=1.0)
    p.update(kw)
    return p


def _empty_links():
    return dict(x=np.zeros(0, np.int32), y=np.zeros(0, np.int32), dir=np.zeros(0, np.int32),
                q=np.zeros(0), ubx=np.zeros(0), uby=np.zeros(0))


def _cat_links(parts):
    if not parts:
        return _empty_links()
    return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}


def wall_candidates(solid, periodic_x, periodic_y):
    """All (x, y, dir) with a fluid x_f whose neighbour along dir is solid.

    Raises ValueError if a fluid node touches a non-periodic edge (the mask must be padded)."""
    ny, nx = solid.shape
    fluid = solid == 0
    xs, ys, ds = [], [], []
    yy, xx = np.nonzero(fluid)
    for d in range(1, 9):
        xn = xx + CX[d]
        yn = yy + CY[d]
        if periodic_x:
            xn = xn % nx
        if periodic_y:
            yn = yn % ny
        outside = (xn < 0) | (xn >= nx) | (yn < 0) | (yn >= ny)
        if outside.any():
            raise ValueError("fluid node on a non-periodic edge: pad the mask with solid")
        hit = solid[yn, xn] != 0
        xs.append(xx[hit]); ys.append(yy[hit]); ds.append(np.full(hit.sum(), d))
    return (np.concatenate(xs).astype(np.int32), np.concatenate(ys).astype(np.int32),
            np.concatenate(ds).astype(np.int32))


def circle_crossing(px, py, dx, dy, radius):
    """Smallest t in (0, 1] with |p + t d| = radius (p relative to the centre).

    Roots of the quadratic |d|^2 t^2 + 2 (p.d) t + (|p|^2 - R^2) = 0 are taken in the
    cancellation-free form; the nearest crossing from x_f is the smallest positive root."""
    a = dx * dx + dy * dy
    b = 2.0 * (px * dx + py * dy)
    c = px * px + py * py - radius * radius
    disc = np.maximum(b * b - 4.0 * a * c, 0.0)
    sq = np.sqrt(disc)
    qq = -0.5 * (b + np.where(b >= 0.0, sq, -sq))
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = qq / a
        t2 = np.where(qq != 0.0, c / qq, np.inf)
    t1 = np.where(t1 > 0.0, t1, np.inf)
    t2 = np.where(t2 > 0.0, t2, np.inf)
    t = np.minimum(t1, t2)
    return np.minimum(t, 1.0)


# ----------------------------------------------------------------------------- channels

def channel(n_fluid_rows, nx=4, gamma=0.3, kn=0.1, ax=1e-6, u_bottom=0.0, u_top=0.0, **kw):
    """Aligned channel (Sec. IV.A.1): rows 0 and ny-1 solid, walls at distance gamma from the
    first and last fluid rows; periodic in x.  H = (n_fluid_rows - 1) + 2 gamma, so fluid row j
    (counted from the bottom fluid row) sits at y = j + gamma above the lower wall."""
    ny = n_fluid_rows + 2
    solid = np.zeros((ny, nx), np.uint8)
    solid[0, :] = 1
    solid[-1, :] = 1
    h = (n_fluid_rows - 1) + 2.0 * gamma
    xs, ys, ds = wall_candidates(solid, 1, 0)
    q = np.full(len(xs), float(gamma))
    ub = np.where(ys == 1, u_bottom, u_top).astype(np.float64)
    links = dict(x=xs, y=ys, dir=ds, q=q, ubx=ub, uby=np.zeros(len(xs)))
    params = base_params(periodic_x=1, periodic_y=0, kn=kn, h=h, ax=ax)
    params.update(kw)
    y_phys = np.arange(n_fluid_rows) + gamma
    meta = dict(kind="channel", H=h, gamma=gamma, y=y_phys, rows=np.arange(1, n_fluid_rows + 1))
    return dict(params=params, solid=solid, links=links, meta=meta)


def poiseuille_config1():
    """Force-driven slip Poiseuille: 20 fluid rows, 4 periodic columns, gamma = 0.3, Kn = 0.1,
    body acceleration 1e-6, rest start."""
    return channel(20, nx=4, gamma=0.3, kn=0.1, ax=1e-6)


# ----------------------------------------------------------------------- inclined walls

def inclined_channel(tan_theta, nx=120, n_ab=16, kn=0.0194, a=1e-6, ny=None, offset=0.3, **kw):
    """Poiseuille channel whose flat walls are inclined at angle theta to the lattice (Sec.
    IV.A.2, Fig. ScheInPois), driven by a body force a along the walls.

    The lattice is doubly periodic and holds a family of identical parallel channels: with
    v = y - x tan(theta) - offset taken modulo ny, fluid is 0 < v < n_ab (n_ab = the vertical
    extent of the channel, the paper's segment AB) and the rest is solid.  nx tan(theta) must be a
    multiple of ny, so that x -> x + nx maps the walls onto themselves; ny defaults to the smallest
    such value that leaves more than 1 + tan(theta) solid rows between channels (so that no link
    of length <= sqrt 2 meets two walls).  Every link's gamma is the exact crossing of the link with
    the wall line.  Perpendicular width H = n_ab cos(theta); the node's distance from the lower
    wall is v cos(theta).  The default offset keeps every node off the walls."""
    t = float(tan_theta)
    rise = nx * t
    if abs(rise - round(rise)) > 1e-9:
        raise ValueError("nx tan(theta) must be an integer")
    rise = int(round(rise))
    if ny is None:
        cands = [d for d in range(1, rise + 1) if rise % d == 0 and d - n_ab > 1.0 + t]
        if not cands:
            raise ValueError("no period leaves enough solid rows")
        ny = min(cands)
    if rise % ny or ny - n_ab <= 1.0 + t:
        raise ValueError(f"ny = {ny} incompatible with nx tan(theta) = {rise} and n_ab = {n_ab}")
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    v = np.mod(yy - xx * t - offset, ny)
    fluid = (v > 0.0) & (v < n_ab)
    solid = (~fluid).astype(np.uint8)
    xs, ys, ds = wall_candidates(solid, 1, 1)
    # v along the link x_f + s c_d, s in [0, 1], without wrapping (it stays within one period)
    v0 = np.mod(ys - xs * t - offset, ny)
    dv = CY[ds] - CX[ds] * t
    v1 = v0 + dv
    lower = v1 <= 0.0
    upper = v1 >= n_ab
    if not np.all(lower ^ upper):
        raise AssertionError("every link must cross exactly one wall")
    q = np.where(lower, (0.0 - v0) / dv, (n_ab - v0) / dv)
    links = dict(x=xs, y=ys, dir=ds, q=q, ubx=np.zeros(len(xs)), uby=np.zeros(len(xs)))
    cos = 1.0 / math.sqrt(1.0 + t * t)
    h = n_ab * cos
    params = base_params(periodic_x=1, periodic_y=1, kn=kn, h=h, ax=a * cos, ay=a * t * cos)
    params.update(kw)
    meta = dict(kind="inclined", tan_theta=t, H=h, n_ab=n_ab, a=a, offset=offset,
                yprime=np.where(fluid, v * cos, np.nan))
    return dict(params=params, solid=solid, links=links, meta=meta)


def inclined_profile(problem, L1, L2, nu):
    """Analytic velocity along the walls at every fluid node (Sec. IV.A.2):
    u_c [4 (y'/H)(1 - y'/H) + 4 L1 Kn + 8 L2 Kn^2], u_c = a H^2 / (8 nu); NaN on solid nodes."""
    m = problem["meta"]
    h, kn = m["H"], problem["params"]["kn"]
    yp = m["yprime"]
    uc = m["a"] * h * h / (8.0 * nu)
    return uc * (4.0 * yp / h * (1.0 - yp / h) + 4.0 * L1 * kn + 8.0 * L2 * kn * kn), uc


# ----------------------------------------------------------------------- circular walls

def annulus(n=132, r1=32.0, r2=64.0, center=None, u_inner=0.01, u_outer=0.0, kn=0.01, **kw):
    """Cylindrical Couette (Sec. IV.B): solid where |x - c| <= r1 or |x - c| >= r2 (closed sets);
    the inner wall turns with tangential speed u_inner, the outer with u_outer (counter-clockwise
    positive).  Kn = lambda / (r2 - r1), so H = r2 - r1."""
    if center is None:
        center = ((n - 1) / 2.0, (n - 1) / 2.0)
    cx, cy = center
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    d2 = (xx - cx) ** 2 + (yy - cy) ** 2
    solid = ((d2 <= r1 * r1) | (d2 >= r2 * r2)).astype(np.uint8)
    xs, ys, ds = wall_candidates(solid, 0, 0)
    px = xs - cx
    py = ys - cy
    dx = CX[ds].astype(np.float64)
    dy = CY[ds].astype(np.float64)
    xn, yn = xs + CX[ds], ys + CY[ds]
    inner = ((xn - cx) ** 2 + (yn - cy) ** 2) <= r1 * r1
    rad = np.where(inner, r1, r2)
    q = circle_crossing(px, py, dx, dy, rad)
    bx = px + q * dx
    by = py + q * dy
    om = np.where(inner, u_inner / r1, u_outer / r2)
    links = dict(x=xs, y=ys, dir=ds, q=q, ubx=-om * by, uby=om * bx)
    params = base_params(periodic_x=0, periodic_y=0, kn=kn, h=r2 - r1)
    params.update(kw)
    meta = dict(kind="annulus", center=(cx, cy), r1=r1, r2=r2, H=r2 - r1, omega1=u_inner / r1,
                omega2=u_outer / r2, inner=inner)
    return dict(params=params, solid=solid, links=links, meta=meta)


def couette_config2(kn):
    """132 x 132 grid, centre (65.5, 65.5), R1 = 32, R2 = 64, inner wall speed 0.01, outer at rest."""
    return annulus(132, 32.0, 64.0, (65.5, 65.5), 0.01, 0.0, kn=kn)


def _min_image(d, n):
    return d - n * np.round(d / n)


def random_cylinders(n=4096, porosity=0.7, rmin=8.0, rmax=24.0, seed=0, gap=2.0, kn=0.05, h=None, ax=1e-6,
                     ny=None, max_attempts=10_000_000):
    """Random non-overlapping circular cylinders on a doubly periodic n x ny lattice.

    Random sequential addition: radius ~ U[rmin, rmax], centre ~ U over the domain, accepted when
    the periodic (minimum-image) surface gap to every placed cylinder is >= gap; stops as soon as the
    node porosity (fraction of fluid nodes) is <= porosity.  A gap of 2 lattice units guarantees
    that no link of length <= sqrt(2) can meet two cylinders, so each link's crossing belongs to
    the cylinder that owns its solid node.  Solid = |x - c| <= R (min image).  Default H = 2 <R>."""
    nx = n
    ny = n if ny is None else ny
    rng = np.random.Generator(np.random.PCG64(seed))
    solid = np.zeros((ny, nx), np.uint8)
    label = np.full((ny, nx), -1, np.int32)
    cell = 2.0 * rmax + gap
    ncx, ncy = max(1, int(nx // cell)), max(1, int(ny // cell))
    grid = {}
    cyl = []
    n_solid = 0
    total = nx * ny
    attempts = 0
    while n_solid / total < 1.0 - porosity:
        attempts += 1
        if attempts > max_attempts:
            raise RuntimeError("cylinder placement did not reach the target porosity")
        r = rng.uniform(rmin, rmax)
        cx = rng.uniform(0.0, nx)
        cy = rng.uniform(0.0, ny)
        gx, gy = int(cx / nx * ncx) % ncx, int(cy / ny * ncy) % ncy
        ok = True
        for ox in (-1, 0, 1):
            for oy in (-1, 0, 1):
                for k in grid.get(((gx + ox) % ncx, (gy + oy) % ncy), ()):
                    qx, qy, qr = cyl[k]
                    ddx = _min_image(cx - qx, nx)
                    ddy = _min_image(cy - qy, ny)
                    if math.hypot(ddx, ddy) < r + qr + gap:
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        k = len(cyl)
        cyl.append((cx, cy, r))
        grid.setdefault((gx, gy), []).append(k)
        x0, x1 = int(math.floor(cx - r)), int(math.ceil(cx + r))
        y0, y1 = int(math.floor(cy - r)), int(math.ceil(cy + r))
        xs = np.arange(x0, x1 + 1)
        ys = np.arange(y0, y1 + 1)
        X, Y = np.meshgrid(xs, ys)
        inside = (X - cx) ** 2 + (Y - cy) ** 2 <= r * r
        Xw, Yw = X[inside] % nx, Y[inside] % ny
        fresh = solid[Yw, Xw] == 0
        n_solid += int(fresh.sum())
        solid[Yw, Xw] = 1
        label[Yw, Xw] = k
    cyl = np.array(cyl, dtype=np.float64).reshape(-1, 3)
    xs, ys, ds = wall_candidates(solid, 1, 1)
    xn = (xs + CX[ds]) % nx
    yn = (ys + CY[ds]) % ny
    k = label[yn, xn]
    px = _min_image(xs - cyl[k, 0], nx)
    py = _min_image(ys - cyl[k, 1], ny)
    q = circle_crossing(px, py, CX[ds].astype(np.float64), CY[ds].astype(np.float64), cyl[k, 2])
    links = dict(x=xs, y=ys, dir=ds, q=q, ubx=np.zeros(len(xs)), uby=np.zeros(len(xs)))
    if h is None:
        h = 2.0 * float(cyl[:, 2].mean()) if len(cyl) else 1.0
    params = base_params(periodic_x=1, periodic_y=1, kn=kn, h=h, ax=ax)
    meta = dict(kind="cylinders", cylinders=cyl, porosity=1.0 - n_solid / total, label=label, seed=seed)
    return dict(params=params, solid=solid, links=links, meta=meta)


def throughput_config3(n=4096, seed=0):
    """4096 x 4096 doubly periodic random cylinder array, porosity 0.7, radii U[8, 24],
    Kn = 0.05 with H = 2 x (mean of U[8, 24]) = 32, body acceleration 1e-6."""
    return random_cylinders(n=n, porosity=0.7, rmin=8.0, rmax=24.0, seed=seed, kn=0.05, h=32.0, ax=1e-6)


def counts(problem):
    """(fluid nodes, sites, links) of a problem."""
    s = problem["solid"]
    return int((s == 0).sum()), int(s.size), int(len(problem["links"]["x"]))


def batched_sweep_config4(seed=1, n_poiseuille=128, n_couette=128, u_target=1e-3):
    """Uneven-instance sweep: slip Poiseuille channels (fluid rows ~ U{16..512}, 4 periodic columns,
    gamma ~ U[0.05, 0.95]) and cylindrical Couette annuli (outer radius ~ U[16, 128] lu, radius ratio
    0.5, grid 2 R2 + 4 with the centre at the grid centre, inner wall speed 0.01), Kn log-uniform in
    [1e-3, 0.1].  The channel force is set per instance so that the centre-line speed of the
    no-slip parabola, a H^2 / (8 nu), is u_target (low Mach at every H and Kn)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sq6pi = math.sqrt(6.0 / math.pi)
    out = []
    for _ in range(n_poiseuille):
        rows = int(rng.integers(16, 513))
        gamma = float(rng.uniform(0.05, 0.95))
        kn = float(10 ** rng.uniform(-3, -1))
        h = (rows - 1) + 2 * gamma
        nu = sq6pi * kn * h / 3.0        # (tau_s - 1/2)/3 with tau_s from Eq. (tKnrela)
        a = 8.0 * nu * u_target / (h * h)
        out.append(channel(rows, nx=4, gamma=gamma, kn=kn, ax=a))
    for _ in range(n_couette):
        r2 = float(rng.uniform(16.0, 128.0))
        kn = float(10 ** rng.uniform(-3, -1))
        n = int(math.ceil(2 * r2)) + 4
        c = (n - 1) / 2.0
        out.append(annulus(n, 0.5 * r2, r2, (c, c), u_inner=0.01, u_outer=0.0, kn=kn))
    return out
