"""Windows of a periodic lattice for sampled parity checks (test helper, not a test module).

After N steps a site's state depends only on the sites within N lattice units.  A window of half-width
h > N around a site, cut out of the lattice and closed by a one-site solid frame, therefore gives
the site's exact state when the oracle steps the window alone: the sites cut off by the frame get
wall links of their own, and the errors those make travel one site per step.  The method itself is
pinned on the CPU (tests/test_window_method.py) against the oracle run on a whole small lattice."""
import numpy as np

from paper_2012_14707_amd import geometry as G


def samples(pb, rng, n_bulk=24, n_wall=24):
    """(x, y) of sampled fluid sites: bulk, with wall links, and on the periodic seams."""
    ny, nx = pb["solid"].shape
    fluid = np.argwhere(pb["solid"] == 0)
    bulk = fluid[rng.choice(len(fluid), n_bulk, replace=False)]
    L = pb["links"]
    k = rng.choice(len(L["x"]), n_wall, replace=False)
    walls = np.stack([L["y"][k], L["x"][k]], axis=1)
    seam = []
    for y, x in ((0, None), (ny - 1, None), (None, 0), (None, nx - 1)):
        line = pb["solid"][y, :] if y is not None else pb["solid"][:, x]
        idx = np.flatnonzero(line == 0)
        i = int(idx[rng.integers(len(idx))])
        seam.append((y, i) if y is not None else (i, x))
    pts = np.concatenate([bulk, walls, np.array(seam)])
    return [(int(x), int(y)) for y, x in pts]


def window(pb, fields, cx, cy, h):
    """The (2h + 1)^2 window of the periodic lattice centred on (cx, cy), inside a one-site solid
    frame, as an oracle problem, and its initial fields."""
    ny, nx = pb["solid"].shape
    w = 2 * h + 1
    ys = (cy - h + np.arange(w)) % ny
    xs = (cx - h + np.arange(w)) % nx
    solid = np.ones((w + 2, w + 2), np.uint8)
    solid[1:-1, 1:-1] = pb["solid"][np.ix_(ys, xs)]
    L = pb["links"]
    site = L["y"].astype(np.int64) * nx + L["x"]
    win = (ys[:, None].astype(np.int64) * nx + xs[None, :]).ravel()
    pick = np.flatnonzero(np.isin(site, win))
    where = {int(s): (i // w, i % w) for i, s in enumerate(win)}
    lx, ly, ld, lq, lu, lv = [], [], [], [], [], []
    have = set()
    for k in pick:
        wy, wx = where[int(site[k])]
        lx.append(wx + 1), ly.append(wy + 1), ld.append(int(L["dir"][k])), lq.append(float(L["q"][k]))
        lu.append(float(L["ubx"][k])), lv.append(float(L["uby"][k]))
        have.add((wy + 1, wx + 1, int(L["dir"][k])))
    # window-edge fluid sites whose neighbour falls in the frame: links of their own
    for y in range(1, w + 1):
        for x in range(1, w + 1):
            if solid[y, x]:
                continue
            for d in range(1, 9):
                yy, xx = y + int(G.CY[d]), x + int(G.CX[d])
                if solid[yy, xx] and (y, x, d) not in have:
                    lx.append(x), ly.append(y), ld.append(d), lq.append(0.5), lu.append(0.0), lv.append(0.0)
    links = {"x": np.array(lx, np.int32), "y": np.array(ly, np.int32), "dir": np.array(ld, np.int32),
             "q": np.array(lq), "ubx": np.array(lu), "uby": np.array(lv)}
    params = dict(pb["params"], nx=w + 2, ny=w + 2, periodic_x=0, periodic_y=0)
    init = []
    for f, rest in zip(fields, (1.0, 0.0, 0.0)):
        a = np.full((w + 2, w + 2), rest)
        a[1:-1, 1:-1] = f[np.ix_(ys, xs)]
        init.append(a)
    return params, solid, links, init
