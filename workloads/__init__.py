"""Seeded synthetic workloads shared by the tests, the bench and the oracle checks.

This module only builds inputs (scene triangles, bodies, source, receivers,
frequencies); it contains none of the field computation.  The paper's own
scenes (rooms of a few metres with PEC balls, an omnidirectional 2 GHz
transmitter; Sec. III-C) are not available, so these stand in for them at the
sizes used for measurement.  Master seed 231010578; every role draws from its
own ``numpy.random.SeedSequence`` child.

Arrays are float32 (what the GPU library consumes); the oracle receives the
same float32 values promoted to float64.
"""
import numpy as np

MASTER_SEED = 231010578
C0 = 299792458.0

ROOM = (10.0, 8.0, 3.0)
TX_ROOM = (5.0, 4.0, 2.5)
RX_HEIGHT = 1.2
CYL_HEIGHT = 1.7


def _rng(*path):
    ss = np.random.SeedSequence(MASTER_SEED)
    for p in path:
        ss = ss.spawn(p + 1)[p]
    return np.random.default_rng(ss)


def empty_scene():
    return dict(tri=np.zeros((0, 3, 3), np.float32), spheres=np.zeros((0, 4), np.float32),
                cylinders=np.zeros((0, 5), np.float32))


# ---------------------------------------------------------------------------
# Config 1: sphere a = 0.5 m, source at (3,0,0), 4096 receivers on r = 3 m.
# ---------------------------------------------------------------------------

def sphere_ring(n_rx=4096, polarisation="hard"):
    phi = 2 * np.pi * (np.arange(n_rx) + 0.5) / n_rx
    rx = np.stack([3 * np.cos(phi), 3 * np.sin(phi), np.zeros(n_rx)], 1).astype(np.float32)
    sc = empty_scene()
    sc["spheres"] = np.array([[0.0, 0.0, 0.0, 0.5]], np.float32)
    # radial electric dipole -> hard polarisation in the receiver plane;
    # dipole normal to the plane -> soft polarisation.
    dip = (1.0, 0.0, 0.0) if polarisation == "hard" else (0.0, 0.0, 1.0)
    tx = dict(pos=np.array([3.0, 0.0, 0.0], np.float32), dipole=np.array(dip, np.float32), amplitude=1.0)
    return dict(name="sphere-a0.5-ring4096-1GHz", scene=sc, tx=tx, rx=rx,
                freqs=np.array([1e9]), phi=phi)


# ---------------------------------------------------------------------------
# Config 2: sphere a = 1 m, source (4,0,0), 256^2 receivers on x = -3 m,
# 64 frequencies 1..6 GHz.
# ---------------------------------------------------------------------------

def sphere_plane(n_side=256, n_f=64, dipole=(0.0, 0.0, 1.0)):
    c = -4 + 8 * (np.arange(n_side) + 0.5) / n_side
    yy, zz = np.meshgrid(c, c, indexing="ij")
    rx = np.stack([np.full(yy.size, -3.0), yy.ravel(), zz.ravel()], 1).astype(np.float32)
    sc = empty_scene()
    sc["spheres"] = np.array([[0.0, 0.0, 0.0, 1.0]], np.float32)
    tx = dict(pos=np.array([4.0, 0.0, 0.0], np.float32), dipole=np.array(dipole, np.float32), amplitude=1.0)
    return dict(name="sphere-a1-plane256x256-64f", scene=sc, tx=tx, rx=rx,
                freqs=np.linspace(1e9, 6e9, n_f))


# ---------------------------------------------------------------------------
# Indoor room (the room, its adjoint workload and the crowd)
# ---------------------------------------------------------------------------

def _quad_grid(origin, u, v, nu, nv):
    """Right triangles tessellating the rectangle origin + [0,1]u + [0,1]v."""
    i, j = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    i, j = i.ravel(), j.ravel()
    p00 = origin + np.outer(i / nu, u) + np.outer(j / nv, v)
    p10 = origin + np.outer((i + 1) / nu, u) + np.outer(j / nv, v)
    p01 = origin + np.outer(i / nu, u) + np.outer((j + 1) / nv, v)
    p11 = origin + np.outer((i + 1) / nu, u) + np.outer((j + 1) / nv, v)
    t1 = np.stack([p00, p10, p11], 1)
    t2 = np.stack([p00, p11, p01], 1)
    return np.concatenate([t1, t2])


def room_shell(edge=0.052):
    """Walls, floor and ceiling of the 10 x 8 x 3 m room (inward faces)."""
    Lx, Ly, Lz = ROOM
    nx, ny, nz = int(round(Lx / edge)), int(round(Ly / edge)), int(round(Lz / edge))
    o = np.zeros(3)
    X, Y, Z = np.array([Lx, 0, 0]), np.array([0, Ly, 0]), np.array([0, 0, Lz])
    faces = [
        _quad_grid(o, X, Y, nx, ny),            # floor
        _quad_grid(o + Z, X, Y, nx, ny),        # ceiling
        _quad_grid(o, X, Z, nx, nz),            # wall y = 0
        _quad_grid(o + Y, X, Z, nx, nz),        # wall y = Ly
        _quad_grid(o, Y, Z, ny, nz),            # wall x = 0
        _quad_grid(o + X, Y, Z, ny, nz),        # wall x = Lx
    ]
    return np.concatenate(faces)


def box_triangles(lo, hi):
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    v = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]])
    f = [(0, 1, 2), (0, 2, 3), (4, 6, 5), (4, 7, 6), (0, 5, 1), (0, 4, 5),
         (1, 6, 2), (1, 5, 6), (2, 7, 3), (2, 6, 7), (3, 4, 0), (3, 7, 4)]
    return v[np.array(f)]


def furniture(n_box=64):
    """Axis-aligned boxes, sizes U(0.3, 2) m per axis, on the floor, inside the room."""
    rng = _rng(3, 0)
    Lx, Ly, _ = ROOM
    boxes = []
    for _ in range(n_box):
        sz = rng.uniform(0.3, 2.0, 3)
        x0 = rng.uniform(0.0, Lx - sz[0])
        y0 = rng.uniform(0.0, Ly - sz[1])
        boxes.append((np.array([x0, y0, 0.0]), np.array([x0 + sz[0], y0 + sz[1], sz[2]])))
    return boxes


def _disc_hits_box(cx, cy, r, lo, hi, margin=0.02):
    qx = min(max(cx, lo[0]), hi[0])
    qy = min(max(cy, lo[1]), hi[1])
    return (cx - qx) ** 2 + (cy - qy) ** 2 <= (r + margin) ** 2


def place_cylinders(n, boxes, rng, tx=TX_ROOM, wall_margin=0.05):
    """Non-overlapping vertical cylinders (humans): a ~ U(0.15, 0.3), h = 1.7 m."""
    Lx, Ly, _ = ROOM
    out = []
    tries = 0
    while len(out) < n:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place cylinders")
        a = rng.uniform(0.15, 0.3)
        cx = rng.uniform(a + wall_margin, Lx - a - wall_margin)
        cy = rng.uniform(a + wall_margin, Ly - a - wall_margin)
        if (cx - tx[0]) ** 2 + (cy - tx[1]) ** 2 <= (a + 0.05) ** 2:
            continue
        if any(_disc_hits_box(cx, cy, a, lo, hi) for lo, hi in boxes):
            continue
        if any((cx - c[0]) ** 2 + (cy - c[1]) ** 2 <= (a + c[4] + 0.02) ** 2 for c in out):
            continue
        out.append((cx, cy, 0.0, CYL_HEIGHT, a))
    return np.array(out, np.float32)


def room_scene(n_cyl, cyl_stream=0, edge=0.052):
    boxes = furniture()
    tri = np.concatenate([room_shell(edge)] + [box_triangles(lo, hi) for lo, hi in boxes]).astype(np.float32)
    cyl = place_cylinders(n_cyl, boxes, _rng(3, 1, cyl_stream))
    sc = dict(tri=tri, spheres=np.zeros((0, 4), np.float32), cylinders=cyl)
    return sc, boxes


def room_grid(n_side, z=RX_HEIGHT):
    Lx, Ly, _ = ROOM
    xs = Lx * (np.arange(n_side) + 0.5) / n_side
    ys = Ly * (np.arange(n_side) + 0.5) / n_side
    xx, yy = np.meshgrid(xs, ys, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), np.full(xx.size, z)], 1).astype(np.float32)


def room_tx():
    return dict(pos=np.array(TX_ROOM, np.float32), dipole=np.array([0.0, 0.0, 1.0], np.float32), amplitude=1.0)


def room(n_side=512, edge=0.052):
    sc, boxes = room_scene(32, 0, edge)
    return dict(name="room10x8x3-200ktri-32cyl-512x512-5/28GHz", scene=sc, tx=room_tx(),
                rx=room_grid(n_side), freqs=np.array([5e9, 28e9]), boxes=boxes)


def room_adjoint(n_side=128, n_f=16, edge=0.052):
    sc, boxes = room_scene(64, 1, edge)
    return dict(name="room10x8x3-200ktri-64cyl-128x128-16f", scene=sc, tx=room_tx(),
                rx=room_grid(n_side), freqs=np.linspace(3.4e9, 3.8e9, n_f), boxes=boxes)


def crowd(n_frames=256, n_pop=64, step=0.05, edge=0.052, rx_range=(1000, 64000)):
    """Dynamic crowd: the indoor room; 64 cylinders random-walk 0.05 m per
    frame (a move that would collide is rejected); frame f uses the first
    n_f ~ U{0..64} of them and n_rx ~ U{1000..64000} uniform receivers at 1.2 m."""
    boxes = furniture()
    tri = np.concatenate([room_shell(edge)] + [box_triangles(lo, hi) for lo, hi in boxes]).astype(np.float32)
    rng = _rng(4, 0)
    pop = place_cylinders(n_pop, boxes, _rng(4, 1)).astype(np.float64)
    Lx, Ly, _ = ROOM
    body_off = [0]
    rx_off = [0]
    cyls, rxs = [], []
    for f in range(n_frames):
        for i in range(n_pop):
            ang = rng.uniform(0, 2 * np.pi)
            nx = pop[i, 0] + step * np.cos(ang)
            ny = pop[i, 1] + step * np.sin(ang)
            a = pop[i, 4]
            ok = (a + 0.05 <= nx <= Lx - a - 0.05) and (a + 0.05 <= ny <= Ly - a - 0.05)
            ok = ok and (nx - TX_ROOM[0]) ** 2 + (ny - TX_ROOM[1]) ** 2 > (a + 0.05) ** 2
            ok = ok and not any(_disc_hits_box(nx, ny, a, lo, hi) for lo, hi in boxes)
            ok = ok and not any((nx - pop[j, 0]) ** 2 + (ny - pop[j, 1]) ** 2 <= (a + pop[j, 4] + 0.02) ** 2
                                for j in range(n_pop) if j != i)
            if ok:
                pop[i, 0], pop[i, 1] = nx, ny
        nb = int(rng.integers(0, n_pop + 1))
        nr = int(rng.integers(rx_range[0], rx_range[1] + 1))
        cyls.append(pop[:nb].copy())
        r = np.stack([rng.uniform(0, Lx, nr), rng.uniform(0, Ly, nr), np.full(nr, RX_HEIGHT)], 1)
        rxs.append(r)
        body_off.append(body_off[-1] + nb)
        rx_off.append(rx_off[-1] + nr)
    return dict(name="crowd-256frames-0..64cyl-1k..64k-rx-8f", tri=tri,
                cylinders=np.concatenate(cyls).astype(np.float32).reshape(-1, 5),
                body_off=np.array(body_off, np.int64), rx=np.concatenate(rxs).astype(np.float32),
                rx_off=np.array(rx_off, np.int64), tx=room_tx(), freqs=np.linspace(3.4e9, 3.8e9, 8))


def to_oracle(scene, tx, rx):
    """float32 inputs -> float64 copies for the oracle (same values)."""
    sc = dict(tri=None if scene.get("tri") is None else np.asarray(scene["tri"], np.float64),
              spheres=np.asarray(scene["spheres"], np.float64),
              cylinders=np.asarray(scene["cylinders"], np.float64))
    t = dict(pos=np.asarray(tx["pos"], np.float64), dipole=np.asarray(tx["dipole"], np.float64),
             amplitude=float(tx["amplitude"]))
    return sc, t, np.asarray(rx, np.float64)


def small_room(n_cyl=8, edge=0.5, n_side=24, freqs=(5e9, 28e9), spheres=False):
    """The indoor room at a coarse tessellation, fewer cylinders and a
    small receiver grid: a parity-test case the oracle finishes in seconds."""
    sc, boxes = room_scene(n_cyl, 7, edge)
    if spheres:
        sc["spheres"] = np.array([[2.0, 6.5, 0.6, 0.35], [8.2, 1.4, 1.0, 0.5]], np.float32)
    return dict(name="room-coarse-%dcyl-%dx%d" % (n_cyl, n_side, n_side), scene=sc, tx=room_tx(),
                rx=room_grid(n_side), freqs=np.asarray(freqs, float), boxes=boxes)


def random_scene(seed, n_cyl=4, n_sph=2, n_box=3, n_rx_side=(11, 9), n_pts=32, n_f=2):
    """A seeded random small room for parity sweeps: a coarse shell, a few
    boxes, cylinders with random base heights, heights and radii, spheres at
    random heights, the source anywhere in the room (below or above the
    bodies' tops), receivers on a grid at a random height plus random points,
    and random frequencies in 1-30 GHz.  Bodies do not overlap each other or
    the boxes, and the source and receivers may be anywhere (inside bodies
    too: those receivers are flagged)."""
    rng = _rng(8, seed)
    Lx, Ly, Lz = ROOM
    boxes = []
    for _ in range(n_box):
        sz = rng.uniform(0.3, 1.5, 3)
        x0, y0 = rng.uniform(0, Lx - sz[0]), rng.uniform(0, Ly - sz[1])
        boxes.append((np.array([x0, y0, 0.0]), np.array([x0 + sz[0], y0 + sz[1], sz[2]])))
    tri = np.concatenate([room_shell(1.0)] + [box_triangles(lo, hi) for lo, hi in boxes]).astype(np.float32)
    discs = []
    cyl, sph = [], []
    tries = 0
    while len(cyl) + len(sph) < n_cyl + n_sph and tries < 100000:
        tries += 1
        a = rng.uniform(0.1, 0.5)
        cx, cy = rng.uniform(a + 0.05, Lx - a - 0.05), rng.uniform(a + 0.05, Ly - a - 0.05)
        if any(_disc_hits_box(cx, cy, a, lo, hi) for lo, hi in boxes):
            continue
        if any((cx - d[0]) ** 2 + (cy - d[1]) ** 2 <= (a + d[2] + 0.05) ** 2 for d in discs):
            continue
        discs.append((cx, cy, a))
        if len(cyl) < n_cyl:
            z0 = rng.uniform(0.0, 0.5)
            cyl.append((cx, cy, z0, rng.uniform(0.8, 2.5 - z0), a))
        else:
            sph.append((cx, cy, rng.uniform(a, Lz - a), a))
    tx = dict(pos=np.array([rng.uniform(0.2, Lx - 0.2), rng.uniform(0.2, Ly - 0.2), rng.uniform(0.3, 2.8)],
                           np.float32),
              dipole=rng.normal(size=3).astype(np.float32), amplitude=1.0)
    nx, ny = n_rx_side
    xs, ys = np.meshgrid(Lx * (np.arange(nx) + 0.5) / nx, Ly * (np.arange(ny) + 0.5) / ny, indexing="ij")
    grid = np.stack([xs.ravel(), ys.ravel(), np.full(xs.size, rng.uniform(0.2, 2.8))], 1)
    pts = np.stack([rng.uniform(0, Lx, n_pts), rng.uniform(0, Ly, n_pts), rng.uniform(0, Lz, n_pts)], 1)
    sc = dict(tri=tri, spheres=np.array(sph, np.float32).reshape(-1, 4),
              cylinders=np.array(cyl, np.float32).reshape(-1, 5))
    return dict(name="random-room-%d" % seed, scene=sc, tx=tx,
                rx=np.concatenate([grid, pts]).astype(np.float32),
                freqs=np.sort(rng.uniform(1e9, 30e9, n_f)), boxes=boxes)

