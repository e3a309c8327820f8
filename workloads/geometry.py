"""Solid masks and cut links with exact wall fractions (inputs of the method).

Conventions (paper, Section 2, link geometry around Eq. (25)):

* A cut link is (x_f, i): x_f is a fluid node, x_r = x_f - e_i is solid, and
  the wall crosses the segment at x_b = x_f - gamma e_i with gamma in (0, 1].
  e_i therefore points from the wall into the fluid.
* Obstacles are closed sets: a node exactly on a surface is solid, so every
  fluid link has gamma in (0, 1].
* gamma is the first crossing met when walking from x_f towards x_r, computed
  in float64 from the closed-form ray/circle, ray/sphere or ray/plane
  intersection.  A link whose segment grazes a second obstacle before
  entering the one that owns x_r keeps the owner's crossing (this cannot
  happen for the plane walls, and for radius >= 8 balls it needs a graze
  depth below 0.03 lattice units).
* Node index n = x + nx*(y + ny*z), x fastest; 2D lattices use nz = 1.
* x boundary kinds: "periodic"; "pressure" (periodic, with a density jump
  applied by the solver where populations cross the x seam); "outflow"
  (column x = 0 must be solid; at x = nx-1 a population moving in -x is
  taken from (nx-1, y - e_y, z - e_z), a zero x-gradient).  y and z are
  always periodic; walls are solid rows/planes of the mask.

Everything here is input generation: no equilibrium, collision, streaming or
boundary-rule arithmetic.
"""

from dataclasses import dataclass, field
import numpy as np

from .velocities import VELOCITIES, dim as lattice_dim

X_BC = ("periodic", "pressure", "outflow")


@dataclass
class Geometry:
    lattice: str
    shape: tuple                    # (nx, ny, nz)
    solid: np.ndarray               # uint8 (N,), 1 = solid
    node: np.ndarray                # int64 (L,) fluid node of each link
    dir: np.ndarray                 # int8 (L,) direction i (wall -> fluid)
    q: np.ndarray                   # float64 (L,) gamma in (0, 1]
    wall_u: np.ndarray              # float64 (L, D) wall velocity phi(x_b)
    tag: np.ndarray                 # int32 (L,) obstacle tag
    x_bc: str = "periodic"
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self):
        return int(np.prod(self.shape))

    @property
    def n_links(self):
        return int(self.node.shape[0])

    @property
    def n_fluid(self):
        return int(self.n_nodes - int(self.solid.sum()))

    @property
    def D(self):
        return lattice_dim(self.lattice)

    @property
    def n_tags(self):
        return int(self.tag.max()) + 1 if self.n_links else 0

    def coords(self):
        nx, ny, nz = self.shape
        n = np.arange(self.n_nodes, dtype=np.int64)
        return n % nx, (n // nx) % ny, n // (nx * ny)

    def with_wall_u(self, wall_u):
        g = Geometry(self.lattice, self.shape, self.solid, self.node, self.dir,
                     self.q, np.ascontiguousarray(wall_u, dtype=np.float64),
                     self.tag, self.x_bc, dict(self.meta))
        return g

    def with_q(self, q):
        return Geometry(self.lattice, self.shape, self.solid, self.node,
                        self.dir, np.ascontiguousarray(q, dtype=np.float64),
                        self.wall_u, self.tag, self.x_bc, dict(self.meta))


# ----------------------------------------------------------------------------
# primitives


class Balls:
    """Disks (2D) or balls (3D), solid inside (closed), periodic images."""

    def __init__(self, centers, radii, tag=1, omega=None):
        self.c = np.asarray(centers, dtype=np.float64)
        self.r = np.asarray(radii, dtype=np.float64)
        self.tag = tag
        # optional rigid rotation (2D): angular speed of each disk about its
        # centre; phi = omega * (-(y_b - c_y), x_b - c_x)
        self.omega = None if omega is None else np.asarray(omega, np.float64)


class HollowBall:
    """Solid outside (closed) a circle/sphere; used for annulus outer walls
    and pipes.  For a pipe the axis direction is ignored by listing only the
    cross-section axes in `axes`."""

    def __init__(self, center, radius, axes, tag=0):
        self.c = np.asarray(center, dtype=np.float64)
        self.r = float(radius)
        self.axes = tuple(axes)
        self.tag = tag


class PlaneWall:
    """Solid half-space along one axis: side = -1 means coordinate <= lo_node
    is solid with the wall plane at `plane` (between lo_node and lo_node+1);
    side = +1 means coordinate >= hi_node solid with the plane below it."""

    def __init__(self, axis, side, node_limit, plane, tag=0, velocity=None):
        self.axis = axis
        self.side = side
        self.limit = node_limit
        self.plane = float(plane)
        self.tag = tag
        self.velocity = velocity


# ----------------------------------------------------------------------------
# core builder


def _min_image(d, length):
    return d - length * np.round(d / length)


def _pull_source(coords, shape, e, x_bc):
    """Node index of x - e (the node a pull of direction e reads), with y, z
    periodic and x handled per x_bc."""
    x, y, z = coords
    nx, ny, nz = shape
    sx = x - e[0]
    if x_bc == "outflow":
        sx = np.where(sx >= nx, nx - 1, sx)
        sx = np.where(sx < 0, 0, sx)
    else:
        sx = np.mod(sx, nx)
    sy = np.mod(y - e[1], ny)
    sz = np.mod(z - (e[2] if len(e) > 2 else 0), nz)
    return sx + nx * (sy + ny * sz)


def build(lattice, shape, balls=(), hollows=(), planes=(), x_bc="periodic",
          meta=None):
    """Rasterise the primitives into a solid mask and list every cut link."""
    assert x_bc in X_BC
    D = lattice_dim(lattice)
    nx, ny, nz = shape
    if D == 2:
        assert nz == 1
    N = nx * ny * nz
    n = np.arange(N, dtype=np.int64)
    x, y, z = n % nx, (n // nx) % ny, n // (nx * ny)
    pos = [x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)]
    L = [float(nx), float(ny), float(nz)]

    solid = np.zeros(N, dtype=bool)
    ball_label = np.full(N, -1, dtype=np.int32)
    ball_sets = list(balls)
    ball_index = []          # (set index, ball index) per global label
    for si, bs in enumerate(ball_sets):
        for bi in range(len(bs.r)):
            c, r = bs.c[bi], bs.r[bi]
            # bounding box in lattice indices, with periodic wrap
            ranges = []
            for a in range(D):
                lo = int(np.floor(c[a] - r)) - 1
                hi = int(np.ceil(c[a] + r)) + 1
                idx = np.arange(lo, hi + 1)
                ranges.append(np.mod(idx, int(L[a])))
            if D == 2:
                ranges.append(np.zeros(1, dtype=np.int64))
            gx, gy, gz = np.meshgrid(ranges[0], ranges[1], ranges[2],
                                     indexing="ij")
            gx, gy, gz = gx.ravel(), gy.ravel(), gz.ravel()
            d2 = _min_image(gx - c[0], L[0]) ** 2 + _min_image(gy - c[1], L[1]) ** 2
            if D == 3:
                d2 = d2 + _min_image(gz - c[2], L[2]) ** 2
            inside = d2 <= r * r
            nn = (gx + nx * (gy + ny * gz))[inside]
            nn = np.unique(nn)
            if np.any(ball_label[nn] >= 0):
                raise ValueError("overlapping balls")
            ball_label[nn] = len(ball_index)
            ball_index.append((si, bi))
            solid[nn] = True

    hollow_masks = []
    for hb in hollows:
        d2 = np.zeros(N)
        for a in hb.axes:
            d2 = d2 + (pos[a] - hb.c[a]) ** 2
        m = d2 >= hb.r * hb.r
        hollow_masks.append(m)
        solid |= m
    plane_masks = []
    for pw in planes:
        coord = (x, y, z)[pw.axis]
        m = coord <= pw.limit if pw.side < 0 else coord >= pw.limit
        plane_masks.append(m)
        solid |= m

    if x_bc == "outflow" and not solid[x == 0].all():
        raise ValueError("outflow x boundary needs a solid column x = 0")

    if ball_index:
        cs = np.array([ball_sets[si].c[bi] for si, bi in ball_index])
        rs = np.array([ball_sets[si].r[bi] for si, bi in ball_index])
        tg = np.array([ball_sets[si].tag for si, bi in ball_index],
                      dtype=np.int32)
    e_all = VELOCITIES[lattice]
    fluid = ~solid
    fl = np.nonzero(fluid)[0]
    link_node, link_dir, link_q, link_u, link_tag = [], [], [], [], []
    for i in range(1, len(e_all)):
        e = e_all[i]
        e3 = np.array([e[0], e[1], e[2] if D == 3 else 0])
        src = _pull_source((x[fl], y[fl], z[fl]), shape, e3, x_bc)
        cut = solid[src]
        if not cut.any():
            continue
        xf = fl[cut]
        xs = src[cut]
        nl = xf.shape[0]
        gamma = np.full(nl, np.inf)
        tag = np.zeros(nl, dtype=np.int32)
        wu = np.zeros((nl, D))
        xf_pos = np.stack([pos[a][xf] for a in range(D)], axis=1)
        ef = e3[:D].astype(np.float64)
        ee = float(ef @ ef)

        def offer(sel, g, t, u):
            # keep the first crossing met along -e_i; ties keep the earlier
            # primitive
            idx = np.nonzero(sel)[0]
            better = g < gamma[idx]
            j = idx[better]
            gamma[j] = g[better]
            tag[j] = t if np.isscalar(t) else np.asarray(t)[better]
            wu[j] = u[better]

        # balls
        lab = ball_label[xs]
        sel = lab >= 0
        if sel.any():
            labs = lab[sel]
            c = cs[labs][:, :D]
            r = rs[labs]
            # offset from the centre of the image that contains x_r = x_f - e
            d = xf_pos[sel] - ef - c
            for a in range(D):
                d[:, a] = _min_image(d[:, a], L[a])
            d = d + ef
            bh = d @ ef
            cc = (d * d).sum(1) - r * r
            disc = bh * bh - ee * cc
            if np.any(cc <= 0) or np.any(disc < 0):
                raise AssertionError("fluid node inside a ball")
            g = cc / (bh + np.sqrt(disc))
            xb = xf_pos[sel] - g[:, None] * ef
            u = np.zeros((g.shape[0], D))
            for k in np.unique(labs):
                si, bi = ball_index[k]
                bs = ball_sets[si]
                if bs.omega is not None and bs.omega[bi] != 0.0:
                    m = labs == k
                    cx, cy = bs.c[bi][0], bs.c[bi][1]
                    u[m, 0] = -bs.omega[bi] * _min_image(xb[m, 1] - cy, L[1])
                    u[m, 1] = bs.omega[bi] * _min_image(xb[m, 0] - cx, L[0])
            offer(sel, g, tg[labs], u)
        # hollow balls (solid outside)
        for hb, m in zip(hollows, hollow_masks):
            sel = m[xs]
            if not sel.any():
                continue
            d = np.zeros((int(sel.sum()), D))
            ea = np.zeros(D)
            for a in hb.axes:
                d[:, a] = xf_pos[sel, a] - hb.c[a]
                ea[a] = ef[a]
            aa = float(ea @ ea)
            bh = d @ ea
            cc = (d * d).sum(1) - hb.r * hb.r
            disc = bh * bh - aa * cc
            if aa == 0 or np.any(cc >= 0):
                raise AssertionError("bad hollow-ball link")
            sq = np.sqrt(disc)
            g = np.where(bh >= 0, (bh + sq) / aa, -cc / (sq - bh))
            offer(sel, g, hb.tag, np.zeros((g.shape[0], D)))
        # plane walls
        for pw, m in zip(planes, plane_masks):
            sel = m[xs]
            if not sel.any():
                continue
            ea = ef[pw.axis]
            if ea == 0:
                raise AssertionError("plane link parallel to the wall")
            g = (xf_pos[sel, pw.axis] - pw.plane) / ea
            u = np.zeros((g.shape[0], D))
            if pw.velocity is not None:
                u[:] = np.asarray(pw.velocity, dtype=np.float64)[:D]
            offer(sel, g, pw.tag, u)
        if not np.all(np.isfinite(gamma)):
            raise AssertionError("cut link without an owning surface")
        if np.any(gamma <= 0) or np.any(gamma > 1 + 1e-12):
            raise AssertionError("gamma outside (0, 1]")
        gamma = np.minimum(gamma, 1.0)
        link_node.append(xf)
        link_dir.append(np.full(nl, i, dtype=np.int8))
        link_q.append(gamma)
        link_u.append(wu)
        link_tag.append(tag)

    if link_node:
        node = np.concatenate(link_node)
        d = np.concatenate(link_dir)
        q = np.concatenate(link_q)
        wu = np.concatenate(link_u)
        tg = np.concatenate(link_tag)
        order = np.lexsort((d, node))
        node, d, q, wu, tg = node[order], d[order], q[order], wu[order], tg[order]
    else:
        node = np.zeros(0, np.int64)
        d = np.zeros(0, np.int8)
        q = np.zeros(0)
        wu = np.zeros((0, D))
        tg = np.zeros(0, np.int32)
    return Geometry(lattice, tuple(int(s) for s in shape),
                    solid.astype(np.uint8), node.astype(np.int64),
                    d.astype(np.int8), np.ascontiguousarray(q),
                    np.ascontiguousarray(wu), tg.astype(np.int32), x_bc,
                    dict(meta or {}))


# ----------------------------------------------------------------------------
# seeded obstacle placement


def place_balls(rng, box, n, rmin, rmax, D, max_tries=2_000_000):
    """Non-overlapping balls with radii ~ U[rmin, rmax] and centres ~ U(box),
    periodic minimum-image separation > r_a + r_b (rejection sampling)."""
    c = np.zeros((n, D))
    r = np.zeros(n)
    k = 0
    tries = 0
    L = np.asarray(box[:D], dtype=np.float64)
    while k < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place %d balls" % n)
        rr = rng.uniform(rmin, rmax)
        cc = rng.uniform(0.0, 1.0, size=D) * L
        if k:
            d = cc[None, :] - c[:k]
            d = d - L * np.round(d / L)
            dist = np.sqrt((d * d).sum(1))
            if np.any(dist <= r[:k] + rr):
                continue
        c[k] = cc
        r[k] = rr
        k += 1
    return c, r


# ----------------------------------------------------------------------------
# named geometries


def annulus(n, u_w, center=(32.3, 31.7), r_in=12.4, r_out=28.6, base=64):
    """Circular Couette cell: inner disk rotating (wall speed u_w), outer
    circle at rest; lengths given for a base x base lattice and scaled by
    n / base."""
    s = n / base
    c = np.array([center[0] * s, center[1] * s, 0.0])
    r1, r2 = r_in * s, r_out * s
    omega = u_w / r1
    inner = Balls([c], [r1], tag=1, omega=[omega])
    outer = HollowBall(c, r2, axes=(0, 1), tag=0)
    return build("D2Q9", (n, n, 1), balls=[inner], hollows=[outer],
                 meta=dict(center=c[:2], r_in=r1, r_out=r2, u_w=u_w))


def poiseuille_channel(ny_mesh, gamma, nx=4, lattice="D2Q9", nz=1):
    """Straight channel of the paper's Poiseuille test: rows j = 0..N_y,
    walls between j = 0 and 1 and between N_y - 1 and N_y at distance
    gamma from the nearest fluid row; x (and z) periodic."""
    ny = ny_mesh + 1
    lo = PlaneWall(1, -1, 0, 1.0 - gamma, tag=0)
    hi = PlaneWall(1, +1, ny_mesh, ny_mesh - 1 + gamma, tag=0)
    return build(lattice, (nx, ny, nz), planes=[lo, hi],
                 meta=dict(gamma=gamma, y_lo=1.0 - gamma,
                           y_hi=ny_mesh - 1 + gamma,
                           H=ny_mesh - 2 + 2 * gamma))


def pipe(radius, nx=4, lattice="D3Q19", center=None, pad=2):
    """Circular pipe along x (Hagen-Poiseuille), cross-section radius in
    lattice units; solid outside the circle (closed)."""
    m = int(np.ceil(2 * radius)) + 2 * pad
    if center is None:
        center = (0.0, (m - 1) / 2.0 + 0.1234, (m - 1) / 2.0 - 0.0567)
    wall = HollowBall(center, radius, axes=(1, 2), tag=0)
    return build(lattice, (nx, m, m), hollows=[wall],
                 meta=dict(center=np.asarray(center), radius=radius))


def random_cylinders(nx, ny, n_obst, rmin, rmax, seed):
    rng = np.random.default_rng(seed)
    c, r = place_balls(rng, (nx, ny), n_obst, rmin, rmax, 2)
    return build("D2Q9", (nx, ny, 1), balls=[Balls(c, r, tag=1)],
                 meta=dict(centers=c, radii=r, seed=seed))


def random_spheres(nx, ny, nz, n_obst, rmin, rmax, seed, x_bc="periodic",
                   lattice="D3Q19"):
    rng = np.random.default_rng(seed)
    c, r = place_balls(rng, (nx, ny, nz), n_obst, rmin, rmax, 3)
    return build(lattice, (nx, ny, nz), balls=[Balls(c, r, tag=1)],
                 x_bc=x_bc, meta=dict(centers=c, radii=r, seed=seed))


def channel_cylinder(nx, ny, radius, center, u_in):
    """Channel flow past one cylinder: solid rows y = 0 and y = ny - 1 (walls
    at y = 1/2 and y = ny - 3/2, tag 0), solid inlet column x = 0 whose wall
    plane x = 1/2 moves at (u_in, 0) (tag 2), cylinder tag 1, zero-gradient
    outflow at x = nx - 1.  Wall rows are listed first so a corner link
    takes the resting wall."""
    walls = [PlaneWall(1, -1, 0, 0.5, tag=0),
             PlaneWall(1, +1, ny - 1, ny - 1.5, tag=0),
             PlaneWall(0, -1, 0, 0.5, tag=2, velocity=(u_in, 0.0))]
    cyl = Balls([np.array([center[0], center[1], 0.0])], [radius], tag=1)
    return build("D2Q9", (nx, ny, 1), balls=[cyl], planes=walls,
                 x_bc="outflow",
                 meta=dict(center=np.asarray(center), radius=radius,
                           u_in=u_in))


def closed_box(nx, ny, nz=1, lattice="D2Q9"):
    """Box with half-way walls on every side (all links gamma = 1/2)."""
    planes = [PlaneWall(0, -1, 0, 0.5), PlaneWall(0, +1, nx - 1, nx - 1.5),
              PlaneWall(1, -1, 0, 0.5), PlaneWall(1, +1, ny - 1, ny - 1.5)]
    if lattice_dim(lattice) == 3:
        planes += [PlaneWall(2, -1, 0, 0.5), PlaneWall(2, +1, nz - 1, nz - 1.5)]
    return build(lattice, (nx, ny, nz), planes=planes)


def empty(lattice, shape, x_bc="periodic"):
    return build(lattice, shape, x_bc=x_bc)
