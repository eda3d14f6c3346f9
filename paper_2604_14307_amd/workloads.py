"""Seeded synthetic workloads (inputs only).

This module builds the initial state that both the GPU library and the CPU
oracle receive: solvent positions and velocities, rigid-body templates (surface
sites in the principal frame, principal moments, mass), body placement,
orientations and momenta.  It performs none of the per-step arithmetic of the
method; it only draws and arranges inputs.

Recipe (the paper's workloads, Sec. II and III; its equilibrated suspension
configurations are not available, so random sequential addition stands in):

* Solvent: uniform positions in the periodic box, Maxwell-Boltzmann velocities
  at kT, mass m, a fixed number density per cell (Sec. II.A: 5 per cell).
* Colloids: spheres whose surface sites lie on a Fibonacci lattice (the paper
  uses a twice-subdivided icosahedron; any discretization is allowed by the
  method, Sec. II.B), site mass 5 (Sec. II.B).  The sites are recentred on
  their centre of mass and rotated into the principal frame, so the inertia
  tensor is diagonal in the body frame.
* Body positions by random sequential addition with a minimum centre distance,
  orientations uniform on SO(3), linear velocities N(0, kT/M), body-frame
  angular momenta N(0, kT I_k).  Total momentum is then removed.
* Solvent particles are stored in the order of their initial (unshifted) cell,
  which is only a choice of labels.
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------------------
# Rigid-body templates

def fibonacci_sphere(nsites: int, radius: float) -> np.ndarray:
    """Sites on a sphere: z_i = 1 - (2i+1)/n, azimuth i * pi * (3 - sqrt 5)."""
    i = np.arange(nsites, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / nsites
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    rxy = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return radius * np.stack([rxy * np.cos(phi), rxy * np.sin(phi), z], axis=1)


def icosphere(radius: float, frequency: int = 4) -> np.ndarray:
    """Sites of a subdivided icosahedron projected onto a sphere: every face
    split into frequency^2 triangles, 10 f^2 + 2 distinct vertices (162 for
    f = 4, the discrete-particle sphere of the paper's single-particle runs)."""
    g = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, g, 0], [1, g, 0], [-1, -g, 0], [1, -g, 0], [0, -1, g], [0, 1, g],
                  [0, -1, -g], [0, 1, -g], [g, 0, -1], [g, 0, 1], [-g, 0, -1], [-g, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1)[:, None]
    # faces: the vertex triples whose pairwise distances are all the edge length
    d = np.linalg.norm(v[:, None] - v[None], axis=2)
    edge = d[d > 1e-9].min()
    adj = np.abs(d - edge) < 1e-9
    faces = [(a, b, c) for a in range(12) for b in range(a + 1, 12) for c in range(b + 1, 12)
             if adj[a, b] and adj[b, c] and adj[a, c]]
    assert len(faces) == 20
    pts = {}
    f = int(frequency)
    for a, b, c in faces:
        for i in range(f + 1):
            for j in range(f + 1 - i):
                k = f - i - j
                p = (i * v[a] + j * v[b] + k * v[c]) / f
                p /= np.linalg.norm(p)
                pts.setdefault(tuple(np.round(p, 12)), p)
    out = np.array(list(pts.values()))
    assert len(out) == 10 * f * f + 2
    return radius * out


def cube_surface(edge: float = 4.0, per_side: int = 5) -> np.ndarray:
    """per_side x per_side grid on each of the 6 faces of a cube (150 sites for 5)."""
    h = 0.5 * edge
    g = (np.arange(per_side) + 0.5) / per_side * edge - h
    u, w = np.meshgrid(g, g, indexing="ij")
    u, w = u.ravel(), w.ravel()
    faces = []
    for axis in range(3):
        for sgn in (-1.0, 1.0):
            f = np.zeros((u.size, 3))
            f[:, axis] = sgn * h
            f[:, (axis + 1) % 3] = u
            f[:, (axis + 2) % 3] = w
            faces.append(f)
    return np.concatenate(faces)


def rod_surface(length: float = 10.0, radius: float = 1.0, rings: int = 18,
                per_ring: int = 10) -> np.ndarray:
    """Open cylinder: rings of sites, odd rings rotated by half a spacing."""
    out = []
    for k in range(rings):
        z = -0.5 * length + (k + 0.5) * length / rings
        off = (math.pi / per_ring) if (k % 2) else 0.0
        ang = off + 2.0 * math.pi * np.arange(per_ring) / per_ring
        out.append(np.stack([radius * np.cos(ang), radius * np.sin(ang), np.full(per_ring, z)], 1))
    return np.concatenate(out)


def dumbbell_surface(radius: float = 1.5, separation: float = 4.0, per_sphere: int = 80):
    s = fibonacci_sphere(per_sphere, radius)
    a = s + np.array([0.0, 0.0, 0.5 * separation])
    b = s - np.array([0.0, 0.0, 0.5 * separation])
    return np.concatenate([a, b])


def rigid_template(sites: np.ndarray, site_mass: float):
    """Recentre sites on their centre of mass and rotate into the principal frame.

    Returns (dhat [S_b,3], principal moments [3], total mass).
    """
    sites = np.asarray(sites, dtype=np.float64)
    m = np.full(sites.shape[0], float(site_mass))
    M = float(m.sum())
    com = (m[:, None] * sites).sum(0) / M
    d = sites - com
    r2 = (d * d).sum(1)
    Itens = (m[:, None, None] * (r2[:, None, None] * np.eye(3)[None] - d[:, :, None] * d[:, None, :])).sum(0)
    evals, evecs = np.linalg.eigh(Itens)
    if np.linalg.det(evecs) < 0:
        evecs[:, 2] = -evecs[:, 2]
    dhat = d @ evecs
    return dhat, evals.copy(), M, m


def random_quaternions(rng, n: int) -> np.ndarray:
    """Uniform unit quaternions (Shoemake), rows (w, x, y, z)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    q = np.stack([np.sqrt(1 - u1) * np.sin(2 * np.pi * u2), np.sqrt(1 - u1) * np.cos(2 * np.pi * u2),
                  np.sqrt(u1) * np.sin(2 * np.pi * u3), np.sqrt(u1) * np.cos(2 * np.pi * u3)], 1)
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def rsa_positions(rng, box, n: int, dmin: float, max_tries: int = 200000000) -> np.ndarray:
    """Random sequential addition of n points, minimum-image distance >= dmin.

    Candidates are drawn in batches and tested against the points accepted
    before the batch with array operations; the survivors are then accepted in
    draw order against the batch's own earlier acceptances.  The points and
    the generator's state afterwards are those of drawing and testing one
    candidate at a time (the unused tail of the last batch is given back by
    rewinding the generator and advancing it past the consumed draws)."""
    box = np.asarray(box, dtype=np.float64)
    ng = np.maximum(1, np.floor(box / dmin).astype(int))
    cw = box / ng
    kcap = 16  # points per grid cell: cells are at least dmin wide, fewer than 2 dmin
    slots = np.full((int(ng[0]), int(ng[1]), int(ng[2]), kcap), -1, dtype=np.int64)
    fill = np.zeros((int(ng[0]), int(ng[1]), int(ng[2])), dtype=np.int64)
    offs = np.array([(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)])
    pts = np.zeros((n, 3))
    d2min = dmin * dmin
    state0 = rng.bit_generator.state
    consumed, placed, tries, batch = 0, 0, 0, 16
    while placed < n:
        cand = rng.random((batch, 3)) * box
        g = np.floor(cand / cw).astype(int) % ng
        nb = (g[:, None, :] + offs[None, :, :]) % ng
        # (candidate, accepted point) pairs in the 27 neighbouring grid cells
        fc = ((nb[..., 0] * ng[1] + nb[..., 1]) * ng[2] + nb[..., 2]).ravel()
        f = fill.ravel()[fc]
        rows = np.repeat(np.arange(len(fc)), f)
        first_of = np.repeat(np.cumsum(f) - f, f)
        pj = slots.reshape(-1)[fc[rows] * kcap + (np.arange(len(rows)) - first_of)]
        ci = rows // len(offs)
        dr = cand[ci] - pts[pj]
        dr -= box * np.round(dr / box)
        conflict = np.zeros(batch, dtype=bool)
        conflict[ci[(dr * dr).sum(-1) < d2min]] = True
        first = placed
        used = batch
        for i in np.flatnonzero(~conflict):
            if first < placed:  # against the points accepted earlier in this batch
                dq = cand[i] - pts[first:placed]
                dq -= box * np.round(dq / box)
                if ((dq * dq).sum(-1) < d2min).any():
                    continue
            gi = tuple(g[i])
            if fill[gi] >= kcap:
                raise RuntimeError("random sequential addition: grid cell over capacity")
            slots[gi + (fill[gi],)] = placed
            fill[gi] += 1
            pts[placed] = cand[i]
            placed += 1
            if placed == n:
                used = int(i) + 1
                break
        tries += used
        consumed += 3 * used
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not converge")
        # about 32 acceptances per batch
        rate = max(placed - first, 1) / used
        batch = int(min(8192, max(16, 32.0 / rate)))
    rng.bit_generator.state = state0
    rng.bit_generator.advance(consumed)
    return pts


def rsa_positions_radii(rng, box, radii, max_tries: int = 200000000) -> np.ndarray:
    """Random sequential addition of spheres of the given radii (no two closer
    than the sum of their radii, minimum image), in the given order."""
    box = np.asarray(box, dtype=np.float64)
    radii = np.asarray(radii, dtype=np.float64)
    n = len(radii)
    cw_min = 2.0 * float(radii.max()) if n else 1.0
    ng = np.maximum(1, np.floor(box / cw_min).astype(int))
    cw = box / ng
    grid: dict = {}
    pts = np.zeros((n, 3))
    tries = 0
    for i in range(n):
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("random sequential addition did not converge")
            p = rng.random(3) * box
            g = np.floor(p / cw).astype(int) % ng
            ok = True
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        key = ((g[0] + dx) % ng[0], (g[1] + dy) % ng[1], (g[2] + dz) % ng[2])
                        for j in grid.get(key, ()):
                            dr = p - pts[j]
                            dr -= box * np.round(dr / box)
                            if dr @ dr < (radii[i] + radii[j]) ** 2:
                                ok = False
                                break
                        if not ok:
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                pts[i] = p
                grid.setdefault((g[0], g[1], g[2]), []).append(i)
                break
    return pts


# ---------------------------------------------------------------------------
# Systems

def srd_params(seed: int, kT_cell: float = 1.0, dt: float = 0.1, alpha_deg: float = 130.0,
               kT: float = 1.0, wca=None, thermalize: int = 1) -> dict:
    a = math.radians(alpha_deg)
    return dict(dt=dt, cos_a=math.cos(a), sin_a=math.sin(a), kT=kT, kT_cell=kT_cell,
                seed=int(seed), thermalize=int(thermalize), wca=dict(wca or {"mode": 0}))


def make_system(ncell, density, templates, centres, quats, rng, kT: float = 1.0,
                a: float = 1.0, m: float = 1.0, n_solvent=None, sort_solvent: bool = True,
                zero_momentum: bool = True) -> dict:
    """Assemble one periodic system.

    templates: list (one per body) of (dhat [S_b,3], I [3], M, site masses [S_b]).
    centres: [B,3] body centres; quats: [B,4] orientations (w,x,y,z).
    """
    ncell = tuple(int(n) for n in ncell)
    L = np.array(ncell, dtype=np.float64) * a
    C = ncell[0] * ncell[1] * ncell[2]
    N = int(round(density * C)) if n_solvent is None else int(n_solvent)
    if sort_solvent and N > 0:
        # uniform positions stored by cell: every particle's cell is drawn
        # uniformly, the cells are laid out in order (a counting sort of the
        # draws), and each particle takes a uniform offset within its cell
        cnt = np.bincount(rng.integers(0, C, N), minlength=C)
        cid = np.repeat(np.arange(C, dtype=np.int64), cnt)
        j = np.stack([cid % ncell[0], (cid // ncell[0]) % ncell[1], cid // (ncell[0] * ncell[1])], axis=1)
        del cid, cnt
        x = (j + rng.random((N, 3))) * a
        del j
    else:
        x = rng.random((N, 3)) * L
    x = np.minimum(x, np.nextafter(L, 0))
    v = rng.normal(0.0, math.sqrt(kT / m), size=(N, 3))

    B = len(templates)
    R = np.zeros((3, B)); q = np.zeros((4, B)); P = np.zeros((3, B)); p = np.zeros((4, B))
    Mv = np.zeros(B); Iv = np.zeros((3, B))
    dh, sm, off = [], [], [0]
    for b, (dhat, I, M, ms) in enumerate(templates):
        R[:, b] = np.asarray(centres[b], dtype=np.float64) % L
        qb = np.asarray(quats[b], dtype=np.float64)
        q[:, b] = qb / np.linalg.norm(qb)
        Mv[b] = M
        Iv[:, b] = I
        P[:, b] = rng.normal(0.0, math.sqrt(kT * M), size=3)
        Lh = rng.normal(0.0, 1.0, size=3) * np.sqrt(kT * np.asarray(I))
        w, xq, yq, zq = q[:, b]
        # conjugate quaternion momentum p = 2 q (x) (0, Lhat)
        p[:, b] = 2.0 * np.array([-xq * Lh[0] - yq * Lh[1] - zq * Lh[2],
                                  w * Lh[0] - zq * Lh[1] + yq * Lh[2],
                                  zq * Lh[0] + w * Lh[1] - xq * Lh[2],
                                  -yq * Lh[0] + xq * Lh[1] + w * Lh[2]])
        dh.append(np.asarray(dhat)); sm.append(np.asarray(ms)); off.append(off[-1] + len(ms))
    if zero_momentum and (N > 0 or B > 0):
        Ptot = m * v.sum(0) + P.sum(1)
        Mtot = m * N + Mv.sum()
        vcm = Ptot / Mtot
        v -= vcm
        P -= Mv[None, :] * vcm[:, None]
    dhat = np.concatenate(dh).T.copy() if B else np.zeros((3, 0))
    return dict(ncell=ncell, a=float(a), m=float(m),
                x=np.ascontiguousarray(x.T), v=np.ascontiguousarray(v.T),
                R=R, img=np.zeros((3, B), dtype=np.int32), q=q, P=P, p=p,
                F=np.zeros((3, B)), T=np.zeros((3, B)), M=Mv, I=Iv,
                site_off=np.array(off, dtype=np.int64), dhat=np.ascontiguousarray(dhat),
                sm=np.concatenate(sm) if B else np.zeros(0))


def sphere_template(radius: float, nsites: int, site_mass: float = 5.0):
    dhat, I, M, ms = rigid_template(fibonacci_sphere(nsites, radius), site_mass)
    return (dhat, I, M, ms)


def single_sphere(ncell=(10, 10, 10), density=5, radius=2.0, nsites=100, site_mass=5.0,
                  centre=None, seed=1, kT=1.0, identity=True):
    """One Fibonacci sphere in a cubic periodic box (the single-particle validation case)."""
    rng = np.random.default_rng(seed)
    L = np.array(ncell, dtype=np.float64)
    centre = 0.5 * L if centre is None else np.asarray(centre, dtype=np.float64)
    tpl = sphere_template(radius, nsites, site_mass)
    quat = np.array([[1.0, 0.0, 0.0, 0.0]]) if identity else random_quaternions(rng, 1)
    return make_system(ncell, density, [tpl], [centre], quat, rng, kT=kT)


def suspension(ncell, density, nbodies, radius=3.0, nsites=200, site_mass=5.0, seed=2, kT=1.0):
    """Hard-sphere suspension: RSA sphere centres at least one diameter apart."""
    rng = np.random.default_rng(seed)
    L = np.array(ncell, dtype=np.float64)
    tpl = sphere_template(radius, nsites, site_mass)
    centres = rsa_positions(rng, L, nbodies, 2.0 * radius) if nbodies else np.zeros((0, 3))
    quats = random_quaternions(rng, nbodies)
    return make_system(ncell, density, [tpl] * nbodies, centres, quats, rng, kT=kT)


# ---------------------------------------------------------------------------
# The five named workloads

def wca_spheres(sigma=6.0, eps=1.0, delta=0.0):
    return {"mode": 1, "eps": eps, "sigma": sigma, "delta": delta}


def sedimentation(params: dict, systems, force=(0.5, 0.0, 0.0)) -> dict:
    """Forced-flow parameters (Sec. III.B): the constant force `force` at every
    body centre and the balancing solvent acceleration g = -B F / (N m), so the
    whole system is force free.  Several systems must share B / N."""
    if isinstance(systems, dict):
        systems = [systems]
    F = np.asarray(force, dtype=np.float64)
    ratios = {(len(s["M"]), s["x"].shape[1], float(s["m"])) for s in systems}
    B, N, m = next(iter(ratios))
    if any(b * N != B * n for b, n, _ in ratios):
        raise ValueError("systems with different body/solvent ratios need different accelerations")
    g = -B * F / (N * m) if N else np.zeros(3)
    return dict(params, f_ext=tuple(float(a) for a in F), g=tuple(float(a) for a in g))


def harmonic_network(dhat: np.ndarray, nneigh: int = 3):
    """Bonds of the harmonic-bond model (Sec. II.B.1) for one template: each
    surface site to its nneigh nearest surface sites (the union of those
    pairs) and to the centre; rest lengths rounded to three decimals, as in the
    paper.  Returns (adjacency lists with rest lengths, centre rest lengths)."""
    d = np.asarray(dhat, dtype=np.float64)
    n = len(d)
    dist = np.sqrt(((d[:, None, :] - d[None, :, :]) ** 2).sum(2))
    np.fill_diagonal(dist, np.inf)
    pairs = set()
    for j in range(n):
        for k in np.argsort(dist[j], kind="stable")[:nneigh]:
            pairs.add((min(j, int(k)), max(j, int(k))))
    adj = [[] for _ in range(n)]
    for a, b in sorted(pairs):
        r0 = round(float(dist[a, b]), 3)
        adj[a].append((b, r0))
        adj[b].append((a, r0))
    adj = [sorted(x) for x in adj]
    rc0 = np.round(np.sqrt((d * d).sum(1)), 3)
    return adj, rc0


def harmonic_from_rigid(wl: dict, kb: float = 5000.0, centre_mass=None, nneigh: int = 3) -> dict:
    """The harmonic-bond model of a rigid workload: the same solvent, the same
    colloids (site positions R + A(q) dhat, rigid-motion velocities
    V + omega x d), a centre site per colloid (mass = site mass unless given),
    and the bond network of harmonic_network."""
    B = wl["M"].shape[0]
    so = np.asarray(wl["site_off"], dtype=np.int64)
    S = int(so[-1])
    L = np.array(wl["ncell"], dtype=np.float64) * float(wl["a"])
    xs = np.zeros((3, S)); vs = np.zeros((3, S))
    xc = np.zeros((3, B)); vc = np.zeros((3, B))
    site_body = np.zeros(S, dtype=np.int32)
    adj_off, adj, adj_r0, rc0 = [0], [], [], np.zeros(S)
    cache = {}
    for b in range(B):
        j0, j1 = int(so[b]), int(so[b + 1])
        dh = wl["dhat"][:, j0:j1].T
        A = quat_matrix(wl["q"][:, b])
        d = dh @ A.T
        V = wl["P"][:, b] / wl["M"][b]
        q, p = wl["q"][:, b], wl["p"][:, b]
        # body-frame angular momentum 1/2 p . P_k q, then omega = A (Lhat / I)
        Lh = 0.5 * np.array([-p[0] * q[1] + p[1] * q[0] + p[2] * q[3] - p[3] * q[2],
                             -p[0] * q[2] - p[1] * q[3] + p[2] * q[0] + p[3] * q[1],
                             -p[0] * q[3] + p[1] * q[2] - p[2] * q[1] + p[3] * q[0]])
        I = wl["I"][:, b]
        w = A @ np.where(I > 0, Lh / np.where(I > 0, I, 1.0), 0.0)
        xs[:, j0:j1] = ((wl["R"][:, b][None, :] + d) % L).T
        vs[:, j0:j1] = (V[None, :] + np.cross(w[None, :], d)).T
        xc[:, b] = wl["R"][:, b] % L
        vc[:, b] = V
        site_body[j0:j1] = b
        key = dh.tobytes()
        if key not in cache:
            cache[key] = harmonic_network(dh, nneigh)
        badj, brc0 = cache[key]
        for jl in range(j1 - j0):
            for k, r0 in badj[jl]:
                adj.append(j0 + k)
                adj_r0.append(r0)
            adj_off.append(len(adj))
        rc0[j0:j1] = brc0
    sm = np.asarray(wl["sm"], dtype=np.float64)
    mc = float(sm[0]) if centre_mass is None and S else float(centre_mass or 1.0)
    return dict(ncell=wl["ncell"], a=wl["a"], m=wl["m"], x=wl["x"], v=wl["v"],
                xs=xs, vs=vs, sm=sm.copy(), site_body=site_body, site_off=so.copy(),
                xc=xc, vc=vc, mc=mc, kb=float(kb), adj_off=np.array(adj_off, dtype=np.int64),
                adj=np.array(adj, dtype=np.int32), adj_r0=np.array(adj_r0), rc0=rc0,
                imgs=np.zeros((3, S), dtype=np.int32), imgc=np.zeros((3, B), dtype=np.int32))


def wca_sites(sigma=1.0, eps=1.0, delta=0.0):
    """WCA between surface sites of different bodies."""
    return {"mode": 2, "eps": eps, "sigma": sigma, "delta": delta}


def quat_matrix(q) -> np.ndarray:
    """Body-to-space rotation of the unit quaternion (w, x, y, z) (placement only)."""
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def rsa_bodies(rng, box, tpls, quats, gap, max_tries: int = 1000000) -> np.ndarray:
    """Random sequential addition of oriented rigid bodies: a trial centre is
    accepted when every site keeps at least `gap` from every site of the bodies
    already placed (minimum image); bounding spheres may interpenetrate."""
    box = np.asarray(box, dtype=np.float64)
    n = len(tpls)
    sites = [tpls[b][0] @ quat_matrix(quats[b]).T for b in range(n)]
    radii = np.array([float(np.sqrt((x ** 2).sum(1)).max()) if len(x) else 0.0 for x in sites])
    reach = 2.0 * float(radii.max()) + gap if n else 1.0
    ng = np.maximum(1, np.floor(box / reach).astype(int))
    cw = box / ng
    grid: dict = {}
    pts = np.zeros((n, 3))
    for i in range(n):
        for _ in range(max_tries):
            p = rng.random(3) * box
            g = np.floor(p / cw).astype(int) % ng
            ok = True
            keys = {((g[0] + dx) % ng[0], (g[1] + dy) % ng[1], (g[2] + dz) % ng[2])
                    for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)}
            for key in keys:
                for j in grid.get(key, ()):
                    dc = p - pts[j]
                    dc -= box * np.round(dc / box)
                    if dc @ dc >= (radii[i] + radii[j] + gap) ** 2:
                        continue
                    d = (sites[i][:, None, :] + dc) - sites[j][None, :, :]
                    d -= box * np.round(d / box)
                    if ((d * d).sum(2) < gap * gap).any():
                        ok = False
                        break
                if not ok:
                    break
            if ok:
                pts[i] = p
                grid.setdefault((g[0], g[1], g[2]), []).append(i)
                break
        else:
            raise RuntimeError("random sequential addition did not converge")
    return pts


def shapes(ncell, density, ncube, nrod, ndumb, site_mass=5.0, seed=5, kT=1.0, gap=2.0 ** (1.0 / 6.0)):
    """Mixed suspension of cubes (edge 4, 150 sites), rods (length 10, radius 1,
    180 sites) and dumbbells (two radius-1.5 spheres 4 apart, 160 sites), shapes
    interleaved, random orientations, placed without overlap: no two sites of
    different bodies closer than `gap` (the site-site WCA cutoff for sigma = 1),
    so no body starts inside another's repulsion."""
    rng = np.random.default_rng(seed)
    kinds = [rigid_template(cube_surface(4.0, 5), site_mass), rigid_template(rod_surface(10.0, 1.0, 18, 10), site_mass),
             rigid_template(dumbbell_surface(1.5, 4.0, 80), site_mass)]
    counts = [ncube, nrod, ndumb]
    order = []
    for i in range(max(counts)):
        for k in range(3):
            if i < counts[k]:
                order.append(k)
    tpls = [kinds[k] for k in order]
    quats = random_quaternions(rng, len(tpls))
    centres = rsa_bodies(rng, np.array(ncell, dtype=np.float64), tpls, quats, gap) if tpls else np.zeros((0, 3))
    return make_system(ncell, density, tpls, centres, quats, rng, kT=kT)


def config(i: int, kT_cell: float = 1.0):
    """Return (workload, params, meta) for named workload i.

    0  single sphere r=2 (100 sites) in 10^3 cells, 5/cell; 100 steps; seed 1
    1  suspension: 60^3 cells, 5/cell, 191 spheres r=3 (200 sites), WCA sigma=6; seed 2
    2  large suspension: 200^3 cells, 10/cell, spheres r=3 at volume fraction 0.3; seed 3
    3  batched: 512 cubic boxes, edge U{12..24}, 5/cell, one sphere r=2 each; seed 4
    4  complex shapes: 128^3 cells, 10/cell, 667 cubes + 667 rods + 666 dumbbells,
       site-site WCA sigma=1; seed 5
    """
    if i == 0:
        wl = single_sphere((10, 10, 10), 5, 2.0, 100, 5.0, centre=(5.0, 5.0, 5.0), seed=1)
        return wl, srd_params(1, kT_cell=kT_cell), dict(name="single sphere 10^3 cells", steps=100)
    if i == 1:
        wl = suspension((60, 60, 60), 5, 191, 3.0, 200, 5.0, seed=2)
        return wl, srd_params(2, kT_cell=kT_cell, wca=wca_spheres()), dict(
            name="hard-sphere suspension 60^3 cells, 1.08M solvent, 191 spheres x 200 sites",
            steps=1000)
    if i == 2:
        vsph = 4.0 / 3.0 * math.pi * 27.0
        nb = int(round(0.3 * 200 ** 3 / vsph))
        wl = suspension((200, 200, 200), 10, nb, 3.0, 200, 5.0, seed=3)
        return wl, srd_params(3, kT_cell=kT_cell, wca=wca_spheres()), dict(
            name="large suspension 200^3 cells, 80M solvent, %d spheres x 200 sites" % nb, steps=200)
    if i == 3:
        return batched_replicas(512, seed=4, kT_cell=kT_cell)
    if i == 4:
        wl = shapes((128, 128, 128), 10, 667, 667, 666, seed=5)
        return wl, srd_params(5, kT_cell=kT_cell, wca=wca_sites()), dict(
            name="complex shapes 128^3 cells, 21M solvent, 667 cubes + 667 rods + 666 dumbbells", steps=500)
    raise ValueError("unknown workload %d" % i)


def paper_benchmark(phi=0.1, seed=6, kT_cell=1.0):
    """The geometry of the paper's rigid-vs-harmonic benchmark (Sec. III.C):
    a cubic box of edge 120, 5 solvent per cell, colloids of diameter 6 at
    volume fraction phi (B = round(phi V / (4/3 pi 3^3))), 162 surface sites of
    mass 5 each (a Fibonacci lattice stands in for the subdivided icosahedron),
    WCA between centres with sigma = 1, Delta = 5 (Eq. (1))."""
    nb = int(round(phi * 120 ** 3 / (4.0 / 3.0 * math.pi * 27.0)))
    wl = suspension((120, 120, 120), 5, nb, 3.0, 162, 5.0, seed=seed)
    par = srd_params(seed, kT_cell=kT_cell, wca=wca_spheres(sigma=1.0, eps=1.0, delta=5.0))
    return wl, par, dict(name="paper benchmark geometry: 120^3 cells, 5/cell (8.64M solvent), phi=%g "
                              "(%d spheres, d=6, 162 sites), WCA sigma=1 Delta=5" % (phi, nb))


def paper_viscosity(phi=0.1, edge=120, seed=7, kT_cell=1.0):
    """The geometry of the paper's reverse nonequilibrium viscosity runs
    (Sec. III.B): a cubic suspension of edge `edge` (RSA spheres of diameter 6,
    162 surface sites of mass 5, WCA sigma = 1, Delta = 5) duplicated along y,
    so the box is edge x 2 edge x edge with 5 solvent per cell, and the
    exchange slabs (width 1) at y = 0 and y = edge.  Returns (workload,
    params, meta, exchange) with exchange = (y0, y1, dy, target, npairs)."""
    rng = np.random.default_rng(seed)
    nb = int(round(phi * edge ** 3 / (4.0 / 3.0 * math.pi * 27.0)))
    half = rsa_positions(rng, np.array([edge, edge, edge], dtype=np.float64), nb, 6.0) if nb else np.zeros((0, 3))
    centres = np.concatenate([half, half + np.array([0.0, float(edge), 0.0])]) if nb else half
    tpl = sphere_template(3.0, 162, 5.0)
    quats = random_quaternions(rng, len(centres))
    wl = make_system((edge, 2 * edge, edge), 5, [tpl] * len(centres), centres, quats, rng)
    par = srd_params(seed, kT_cell=kT_cell, wca=wca_spheres(sigma=1.0, eps=1.0, delta=5.0))
    meta = dict(name="paper viscosity geometry: %d x %d x %d cells, 5/cell (%d solvent), phi=%g "
                     "(%d spheres, d=6, 162 sites), WCA sigma=1 Delta=5; slabs y=0 and y=%d, 100 pairs"
                     % (edge, 2 * edge, edge, wl["x"].shape[1], phi, len(centres), edge))
    return wl, par, meta, (0.0, float(edge), 1.0, 0.5, 100)


def paper_single_sphere(edge=90, nrep=1, seed=12, kT_cell=1.0):
    """The paper's single-particle validation (Sec. III.A): a cubic periodic box
    of edge `edge`, 5 solvent per cell, one sphere of diameter 6 made of the 162
    sites of a subdivided icosahedron (mass 5 each) at the box centre, randomly
    oriented; nrep independent replicas advanced together."""
    tpl = rigid_template(icosphere(3.0, 4), 5.0)
    systems = []
    for r in range(nrep):
        rng = np.random.default_rng([seed, r])
        c = 0.5 * edge
        systems.append(make_system((edge, edge, edge), 5, [tpl], [(c, c, c)], random_quaternions(rng, 1), rng))
    return systems, srd_params(seed, kT_cell=kT_cell), dict(
        name="single sphere (162-site icosahedron, d=6) in %d^3 cells, 5/cell, %d replica(s)" % (edge, nrep))


def batched_replicas(nrep=512, seed=4, lo=12, hi=24, density=5, kT_cell=1.0):
    """Independent cubic boxes with integer edges drawn uniformly from lo..hi."""
    rng = np.random.default_rng(seed)
    edges = rng.integers(lo, hi + 1, size=nrep)
    tpl = sphere_template(2.0, 100, 5.0)
    systems = []
    for r in range(nrep):
        n = int(edges[r])
        rr = np.random.default_rng([seed, r])
        systems.append(make_system((n, n, n), density, [tpl], [(0.5 * n, 0.5 * n, 0.5 * n)],
                                   np.array([[1.0, 0.0, 0.0, 0.0]]), rr))
    return systems, srd_params(seed, kT_cell=kT_cell), dict(
        name="%d replicas, edges %d..%d cells, 5/cell, one sphere r=2 each" % (nrep, lo, hi),
        steps=10000)
