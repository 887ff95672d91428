"""Seeded synthetic scene generators shared by the oracle and the GPU path.

This module only *describes* geometry: point clouds in a body frame (or in
the lab frame for fixed boundaries), surface/arc-length quadrature weights,
travelling-wave parameters and initial rigid-body states.  It holds none of
the method's arithmetic: no stokeslet, no nearest-neighbour map, no
assembly, no solve and no evaluation of the geometry at a time t.  Both the
oracle and the HIP path consume the arrays produced here and evaluate
everything else on their own.

Scene dictionary (all arrays numpy, float64 unless stated, int32 indices):

  eps, mu            regularisation parameter and viscosity
  N, Q, M, G         coarse points, quadrature points, free bodies, NN groups
  xi   (3, N)        coarse points: body-frame offset (free bodies) or lab
                     position (fixed points, body == -1)
  body (N,) int32    -1 = fixed point with prescribed velocity, else 0..M-1
  part (N,) int32    travelling-wave part index, -1 = rigid offset only
  s    (N,)          arc parameter used by wave parts
  ufix (3, N)        prescribed lab velocity of fixed points (0 elsewhere)
  Xi, bodyX, partX, sX  the same for the Q quadrature points
  w0   (Q,)          quadrature weight; multiplied by |d xi/ds| on wave parts
  group_off (G+1,) int32  coarse points of NN group g are group_off[g]..[g+1]
  groupX (Q,) int32  NN group of each quadrature point
  wave (P, 6)        per part: beta, A0, A1, k, omega, phi; the body-frame
                     displacement of a wave point is
                     (beta*s, (A0 + A1*s)*sin(k*s - omega*t + phi), 0)
  Y0   (M, 12)       initial state per body: origin x0 (3) then the body
                     frame B (3x3, row-major; column i is body axis i)
  ftext (M, 6)       external force and torque on each free body

All generators use numpy.random.default_rng(seed).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "sphere_scene",
    "filament_scene",
    "sperm_channel_scene",
    "rod_wall_scene",
    "rod_wall_batch",
    "random_rotation",
    "scene_sizes",
]


# ----------------------------------------------------------------------------
# point-cloud helpers (geometry of the inputs only)
# ----------------------------------------------------------------------------

def _cube_face_frames():
    """Six cube faces as (normal, tangent1, tangent2) unit vectors."""
    e = np.eye(3)
    faces = []
    for ax in range(3):
        for sgn in (1.0, -1.0):
            n = sgn * e[ax]
            t1 = e[(ax + 1) % 3]
            t2 = e[(ax + 2) % 3]
            faces.append((n, t1, t2))
    return faces


def _solid_angle_corner(x, y):
    return np.arctan(x * y / np.sqrt(1.0 + x * x + y * y))


def cube_sphere(n, a=1.0, centre=(0.0, 0.0, 0.0)):
    """Cell-centred n x n grid on each cube face, radially projected to a
    sphere of radius a.  Returns points (3, 6n^2) and exact spherical cell
    areas (6n^2,) from the solid angle of each face cell."""
    edges = np.linspace(-1.0, 1.0, n + 1)
    mids = 0.5 * (edges[:-1] + edges[1:])
    pts, wts = [], []
    for nrm, t1, t2 in _cube_face_frames():
        for i in range(n):
            for j in range(n):
                p = nrm + mids[i] * t1 + mids[j] * t2
                pts.append(a * p / np.linalg.norm(p))
                x1, x2, y1, y2 = edges[i], edges[i + 1], edges[j], edges[j + 1]
                om = (_solid_angle_corner(x2, y2) - _solid_angle_corner(x1, y2)
                      - _solid_angle_corner(x2, y1) + _solid_angle_corner(x1, y1))
                wts.append(a * a * om)
    P = np.array(pts).T + np.asarray(centre, dtype=np.float64)[:, None]
    return np.ascontiguousarray(P), np.array(wts)


def fibonacci_ellipsoid(count, semi_axes):
    """Golden-spiral lattice on the unit sphere mapped to an ellipsoid with
    the given semi-axes; weights are the mapped area elements so that they
    sum to (approximately) the ellipsoid's surface area."""
    a, b, c = semi_axes
    i = np.arange(count, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / count
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    p = np.stack([r * np.cos(phi), r * np.sin(phi), z])
    P = np.stack([a * p[0], b * p[1], c * p[2]])
    scale = np.sqrt((p[0] / a) ** 2 + (p[1] / b) ** 2 + (p[2] / c) ** 2)
    w = (4.0 * math.pi / count) * a * b * c * scale
    return np.ascontiguousarray(P), w


def box_walls(lengths, h, sub=4):
    """Six faces of an axis-aligned box centred at the origin, each covered
    by a uniform cell-centred grid of spacing h (coarse) and by sub x sub
    sub-cells per coarse cell (fine).  Returns coarse points, fine points,
    fine weights."""
    L = np.asarray(lengths, dtype=np.float64)
    cpts, fpts, fw = [], [], []
    for ax in range(3):
        a1, a2 = (ax + 1) % 3, (ax + 2) % 3
        n1 = int(round(L[a1] / h))
        n2 = int(round(L[a2] / h))
        h1, h2 = L[a1] / n1, L[a2] / n2
        for sgn in (1.0, -1.0):
            for i in range(n1):
                for j in range(n2):
                    c = np.zeros(3)
                    c[ax] = sgn * L[ax] / 2
                    c[a1] = -L[a1] / 2 + (i + 0.5) * h1
                    c[a2] = -L[a2] / 2 + (j + 0.5) * h2
                    cpts.append(c)
                    for ii in range(sub):
                        for jj in range(sub):
                            f = c.copy()
                            f[a1] = -L[a1] / 2 + i * h1 + (ii + 0.5) * h1 / sub
                            f[a2] = -L[a2] / 2 + j * h2 + (jj + 0.5) * h2 / sub
                            fpts.append(f)
                            fw.append(h1 * h2 / (sub * sub))
    return (np.ascontiguousarray(np.array(cpts).T), np.ascontiguousarray(np.array(fpts).T),
            np.array(fw))


def plane_patch(k, side, centre=(0.0, 0.0, 0.0), sub=4):
    """k x k cell-centred grid on the square z = centre[2] of the given side,
    with sub x sub sub-cells per cell as quadrature points."""
    h = side / k
    cx, cy, cz = centre
    e = -side / 2 + (np.arange(k) + 0.5) * h
    gx, gy = np.meshgrid(e, e, indexing="ij")
    C = np.stack([gx.ravel() + cx, gy.ravel() + cy, np.full(k * k, cz)])
    f = -side / 2 + (np.arange(k * sub) + 0.5) * (h / sub)
    fx, fy = np.meshgrid(f, f, indexing="ij")
    F = np.stack([fx.ravel() + cx, fy.ravel() + cy, np.full(k * k * sub * sub, cz)])
    w = np.full(F.shape[1], (h / sub) ** 2)
    return np.ascontiguousarray(C), np.ascontiguousarray(F), w


def random_rotation(rng):
    """Uniformly distributed rotation matrix from a random unit quaternion
    (Shoemake's subgroup algorithm)."""
    u1, u2, u3 = rng.random(3)
    q = np.array([
        math.sqrt(1 - u1) * math.sin(2 * math.pi * u2),
        math.sqrt(1 - u1) * math.cos(2 * math.pi * u2),
        math.sqrt(u1) * math.sin(2 * math.pi * u3),
        math.sqrt(u1) * math.cos(2 * math.pi * u3),
    ])
    x, y, z, w = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


# ----------------------------------------------------------------------------
# scene assembly
# ----------------------------------------------------------------------------

class _Builder:
    """Accumulates coarse/fine point blocks group by group."""

    def __init__(self, eps, mu):
        self.eps, self.mu = float(eps), float(mu)
        self.c = []   # (xi, body, part, s, ufix)
        self.f = []   # (Xi, body, part, s, w0, group)
        self.group_sizes = []
        self.wave = []
        self.Y0 = []
        self.ftext = []

    def add_wave(self, beta, A0, A1, k, omega, phi):
        self.wave.append([beta, A0, A1, k, omega, phi])
        return len(self.wave) - 1

    def add_body(self, x0, B, ft=None):
        self.Y0.append(np.concatenate([np.asarray(x0, float), np.asarray(B, float).ravel()]))
        self.ftext.append(np.zeros(6) if ft is None else np.asarray(ft, float))
        return len(self.Y0) - 1

    def add_group(self, blocks_c, blocks_f):
        """blocks_c / blocks_f: lists of dicts with keys pts, body, part, s,
        (ufix) / (w0); all blocks form one nearest-neighbour group."""
        g = len(self.group_sizes)
        n = 0
        for b in blocks_c:
            cnt = b["pts"].shape[1]
            self.c.append((b["pts"], np.full(cnt, b["body"], np.int32),
                           np.full(cnt, b.get("part", -1), np.int32),
                           np.asarray(b.get("s", np.zeros(cnt)), float),
                           np.asarray(b.get("ufix", np.zeros((3, cnt))), float)))
            n += cnt
        for b in blocks_f:
            cnt = b["pts"].shape[1]
            self.f.append((b["pts"], np.full(cnt, b["body"], np.int32),
                           np.full(cnt, b.get("part", -1), np.int32),
                           np.asarray(b.get("s", np.zeros(cnt)), float),
                           np.asarray(b["w0"], float), np.full(cnt, g, np.int32)))
        self.group_sizes.append(n)
        return g

    def build(self, **meta):
        xi = np.concatenate([c[0] for c in self.c], axis=1)
        Xi = np.concatenate([f[0] for f in self.f], axis=1)
        go = np.zeros(len(self.group_sizes) + 1, np.int32)
        go[1:] = np.cumsum(self.group_sizes)
        M = len(self.Y0)
        sc = dict(
            eps=self.eps, mu=self.mu,
            N=int(xi.shape[1]), Q=int(Xi.shape[1]), M=M, G=len(self.group_sizes),
            xi=np.ascontiguousarray(xi),
            body=np.concatenate([c[1] for c in self.c]),
            part=np.concatenate([c[2] for c in self.c]),
            s=np.concatenate([c[3] for c in self.c]),
            ufix=np.ascontiguousarray(np.concatenate([c[4] for c in self.c], axis=1)),
            Xi=np.ascontiguousarray(Xi),
            bodyX=np.concatenate([f[1] for f in self.f]),
            partX=np.concatenate([f[2] for f in self.f]),
            sX=np.concatenate([f[3] for f in self.f]),
            w0=np.concatenate([f[4] for f in self.f]),
            groupX=np.concatenate([f[5] for f in self.f]),
            group_off=go,
            wave=np.array(self.wave, float).reshape(-1, 6),
            Y0=np.array(self.Y0, float).reshape(M, 12),
            ftext=np.array(self.ftext, float).reshape(M, 6),
        )
        sc.update(meta)
        return sc


def sphere_scene(nc=4, nq=16, a=1.0, eps=0.01, mu=1.0, U=(1.0, 0.0, 0.0),
                 Omega=(0.0, 0.0, 0.0), free=False, force=None, torque=None):
    """Unit sphere resistance problem on a cube-to-sphere projected grid:
    6*nc^2 force points and 6*nq^2 quadrature points with exact spherical
    cell areas.  Fixed (resistance) form: prescribed rigid velocity
    U + Omega x r.  free=True gives a one-body mobility problem instead, with
    the given external force and torque."""
    xc, _ = cube_sphere(nc, a)
    xq, wq = cube_sphere(nq, a)
    bld = _Builder(eps, mu)
    if free:
        body = bld.add_body(np.zeros(3), np.eye(3),
                            np.concatenate([np.zeros(3) if force is None else force,
                                            np.zeros(3) if torque is None else torque]))
        bld.add_group([dict(pts=xc, body=body)], [dict(pts=xq, body=body, w0=wq)])
    else:
        U = np.asarray(U, float)
        Om = np.asarray(Omega, float)
        ufix = U[:, None] + np.cross(Om[None, :], xc.T).T
        bld.add_group([dict(pts=xc, body=-1, ufix=ufix)], [dict(pts=xq, body=-1, w0=wq)])
    return bld.build(name=f"sphere_nc{nc}_nq{nq}", a=a)


def filament_scene(M=1, seed=0, Nf=40, Qf=400, eps=0.01, mu=1.0, amp=0.1,
                   phase_random=False, spacing=1.5):
    """M undulating filaments of unit body length.  Body-frame centreline
    (s - 1/2, amp*sin(2*pi*s - t + phi), 0), s in [0, 1]; force points at
    s_n = (n+1/2)/Nf, quadrature points at s_q = (q+1/2)/Qf with weight
    |d xi/ds| / Qf.  Centres are rejection-sampled in a cube of side
    1.5*ceil(M^(1/3)) + 1 with pairwise distance >= spacing; orientations
    are uniform random rotations."""
    rng = np.random.default_rng(seed)
    side = 1.5 * math.ceil(M ** (1.0 / 3.0) - 1e-12) + 1.0
    centres = []
    tries = 0
    while len(centres) < M:
        c = (rng.random(3) - 0.5) * side
        tries += 1
        if all(np.linalg.norm(c - d) >= spacing for d in centres):
            centres.append(c)
        if tries > 100000:
            raise RuntimeError("could not place filaments")
    bld = _Builder(eps, mu)
    sN = (np.arange(Nf) + 0.5) / Nf
    sQ = (np.arange(Qf) + 0.5) / Qf
    for b in range(M):
        R = random_rotation(rng)
        phi = rng.random() * 2 * math.pi if phase_random else 0.0
        body = bld.add_body(centres[b], R)
        part = bld.add_wave(1.0, amp, 0.0, 2 * math.pi, 1.0, phi)
        base_c = np.zeros((3, Nf)); base_c[0] = -0.5
        base_f = np.zeros((3, Qf)); base_f[0] = -0.5
        bld.add_group([dict(pts=base_c, body=body, part=part, s=sN)],
                      [dict(pts=base_f, body=body, part=part, s=sQ, w0=np.full(Qf, 1.0 / Qf))])
    return bld.build(name=f"filaments_M{M}_seed{seed}")


def sperm_channel_scene(K=10, h=1.0 / 16, seed=0, eps=0.01, mu=1.0,
                        head_axes=(0.02, 0.016, 0.01), Nh=100, Qh=1600, Nf=40, Qf=400,
                        box=(4.0, 1.0, 0.5)):
    """K sperm-like swimmers (ellipsoidal head + flagellum, one rigid frame
    each) in a closed rectangular channel.  The flagellum's body-frame
    centreline is (-a_h - s, 0.2*s*sin(3*pi*s - t + phi), 0).  Swimmers sit
    on a 3 x 2 x 7 lattice of slots (seeded choice, small jitter), heading
    +x.  Each channel face is a grid of spacing h with 4 x 4 quadrature
    sub-cells per cell; the channel is one nearest-neighbour group and
    each swimmer another."""
    rng = np.random.default_rng(seed)
    slots = [(x, y, z) for x in (-1.3, 0.0, 1.3) for y in (-0.25, 0.25)
             for z in np.round(np.arange(-0.18, 0.18 + 1e-9, 0.06), 10)]
    if K > len(slots):
        raise ValueError("too many swimmers for the slot lattice")
    order = rng.permutation(len(slots))[:K]
    ah = head_axes[0]
    hc, _ = fibonacci_ellipsoid(Nh, head_axes)
    hq, hw = fibonacci_ellipsoid(Qh, head_axes)
    sN = (np.arange(Nf) + 0.5) / Nf
    sQ = (np.arange(Qf) + 0.5) / Qf
    bld = _Builder(eps, mu)
    for i in order:
        x, y, z = slots[i]
        c = np.array([x + (rng.random() - 0.5) * 0.1, y, z + (rng.random() - 0.5) * 0.01])
        phi = rng.random() * 2 * math.pi
        body = bld.add_body(c, np.eye(3))
        part = bld.add_wave(-1.0, 0.0, 0.2, 3 * math.pi, 1.0, phi)
        fc = np.zeros((3, Nf)); fc[0] = -ah
        fq = np.zeros((3, Qf)); fq[0] = -ah
        bld.add_group([dict(pts=hc, body=body), dict(pts=fc, body=body, part=part, s=sN)],
                      [dict(pts=hq, body=body, w0=hw),
                       dict(pts=fq, body=body, part=part, s=sQ, w0=np.full(Qf, 1.0 / Qf))])
    wc, wq, ww = box_walls(box, h)
    bld.add_group([dict(pts=wc, body=-1)], [dict(pts=wq, body=-1, w0=ww)])
    return bld.build(name=f"sperm_K{K}_h{round(1 / h)}_seed{seed}")


def rod_wall_scene(n_target, rng, eps=0.005, mu=1.0, rod_len=0.5, Nr=20, Qr=200,
                   patch_side=2.0):
    """Resistance problem: a rigid rod of length rod_len tilted from the wall
    normal, rotating with Omega = (0, 0, 1) about the normal through its
    base, over a no-slip square plane patch; the patch has k x k cells with
    k = round(sqrt(N_w)), N_w = max(80, round(n_target/3) - 20)."""
    Nw = max(80, int(round(n_target / 3.0)) - 20)
    k = max(1, int(round(math.sqrt(Nw))))
    theta = rng.random() * math.radians(40.0)
    az = rng.random() * 2 * math.pi
    d = np.array([math.sin(theta) * math.cos(az), math.sin(theta) * math.sin(az), math.cos(theta)])
    base = np.array([0.0, 0.0, 2 * eps])
    sN = (np.arange(Nr) + 0.5) / Nr * rod_len
    sQ = (np.arange(Qr) + 0.5) / Qr * rod_len
    rc = base[:, None] + d[:, None] * sN[None, :]
    rq = base[:, None] + d[:, None] * sQ[None, :]
    Om = np.array([0.0, 0.0, 1.0])
    urc = np.cross(Om[None, :], (rc - base[:, None]).T).T
    wc, wq, ww = plane_patch(k, patch_side)
    bld = _Builder(eps, mu)
    bld.add_group([dict(pts=rc, body=-1, ufix=urc)],
                  [dict(pts=rq, body=-1, w0=np.full(Qr, rod_len / Qr))])
    bld.add_group([dict(pts=wc, body=-1)], [dict(pts=wq, body=-1, w0=ww)])
    return bld.build(name=f"rodwall_n{n_target}", theta=theta, azimuth=az)


def rod_wall_batch(B=512, seed=0, lo=300, hi=6000):
    """B independent rod-over-wall resistance problems whose target sizes
    are drawn log-uniformly in [lo, hi] unknowns."""
    rng = np.random.default_rng(seed)
    targets = np.exp(rng.uniform(math.log(lo), math.log(hi), size=B))
    return [rod_wall_scene(int(round(t)), rng) for t in targets]


def tracer_grid(nx, ny, xr, yr, z):
    """nx x ny tracers on a rectangular grid (end points included) spanning
    xr x yr in the plane z = const; returns (3, nx*ny), x fastest."""
    gx = np.linspace(xr[0], xr[1], nx)
    gy = np.linspace(yr[0], yr[1], ny)
    X, Y = np.meshgrid(gx, gy, indexing="xy")
    return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel(), np.full(nx * ny, float(z))]))


def scene_sizes(sc):
    """(N, Q, M, n) with n = 3N + 6M unknowns."""
    return sc["N"], sc["Q"], sc["M"], 3 * sc["N"] + 6 * sc["M"]
