"""Seeded synthetic scenes and shading-point sets.

This module only builds inputs: triangle soups with vertex normals, point
emitters, a planar receiver and query points.  It holds none of the caustic
method's arithmetic and is shared by the FP64 oracle tests and the HIP path.

Layout (structure of arrays, float32, the canonical precision of every input):

* ``pos``  [9, n]  rows p0.x p0.y p0.z p1.x ... p2.z of each specular triangle
* ``nrm``  [9, n]  the three vertex normals in the same order
* ``epos`` [3, ne] point-emitter positions, ``eI`` [ne] intensities
* ``q0, f1, f2`` [3] the receiver parallelogram x = q0 + u f1 + v f2,
  (u, v) in [0, 1]^2 (the receiver's texture space)
* ``chain`` "R" (one reflection), "T" (one refraction) or "RR" (two
  reflections, second surface in ``pos2``/``nrm2``); ``eta`` is the ratio of
  indices of refraction eta' for "T" (incident side over transmitted side).

The scenes follow the workload shapes of the paper's evaluation (single
reflection off curved tessellated casters, refraction through a water
surface, two specular bounces between facing surfaces); the paper's own
scenes are not available, so these seeded stand-ins replace them.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 2504_19163


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _normalize(v, axis=0):
    return v / np.linalg.norm(v, axis=axis, keepdims=True)


def _scene(chain, pos, nrm, epos, eI, q0, f1, f2, eta=1.0, pos2=None, nrm2=None, name=""):
    s = {
        "name": name,
        "chain": chain,
        "pos": _f32(pos),
        "nrm": _f32(nrm),
        "epos": _f32(np.asarray(epos).reshape(3, -1)),
        "eI": _f32(np.asarray(eI).reshape(-1)),
        "q0": _f32(q0),
        "f1": _f32(f1),
        "f2": _f32(f2),
        "eta": float(np.float32(eta)),
    }
    if pos2 is not None:
        s["pos2"] = _f32(pos2)
        s["nrm2"] = _f32(nrm2)
    return s


def _grid_triangles(X, Y, Z, N):
    """Split every cell of a (m+1)x(m+1) vertex grid into two triangles that are
    counter-clockwise when seen from +z.  X, Y, Z, N are vertex arrays
    ([m+1, m+1] for X/Y/Z, [3, m+1, m+1] for N)."""
    m = X.shape[0] - 1
    P = np.stack([X, Y, Z])  # [3, m+1, m+1], index [.., i(x), j(y)]
    a = (slice(None), slice(0, m), slice(0, m))
    b = (slice(None), slice(1, m + 1), slice(0, m))
    c = (slice(None), slice(0, m), slice(1, m + 1))
    d = (slice(None), slice(1, m + 1), slice(1, m + 1))
    tris_p, tris_n = [], []
    for (i0, i1, i2) in ((a, b, c), (b, d, c)):
        tris_p.append(np.concatenate([P[i0].reshape(3, -1), P[i1].reshape(3, -1), P[i2].reshape(3, -1)]))
        tris_n.append(np.concatenate([N[i0].reshape(3, -1), N[i1].reshape(3, -1), N[i2].reshape(3, -1)]))
    # interleave the two triangles of each cell so triangle 2k and 2k+1 share a cell
    pos = np.stack(tris_p, axis=2).reshape(9, -1)
    nrm = np.stack(tris_n, axis=2).reshape(9, -1)
    return pos, nrm


def _sinusoid_heightfield(m, lo, hi, amp, rng, n_waves=4, fmin=1.0, fmax=4.0):
    """z = amp * sum_s sin(pi f_s (x cos th_s + y sin th_s) + ph_s) with analytic
    normals (-dz/dx, -dz/dy, 1)/|.|, sampled on an (m+1)^2 vertex grid."""
    f = rng.uniform(fmin, fmax, n_waves)
    th = rng.uniform(0, 2 * math.pi, n_waves)
    ph = rng.uniform(0, 2 * math.pi, n_waves)
    xs = np.linspace(lo, hi, m + 1)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    Z = np.zeros_like(X)
    dZx = np.zeros_like(X)
    dZy = np.zeros_like(X)
    for s in range(n_waves):
        k = math.pi * f[s]
        arg = k * (X * math.cos(th[s]) + Y * math.sin(th[s])) + ph[s]
        Z += amp * np.sin(arg)
        dZx += amp * np.cos(arg) * k * math.cos(th[s])
        dZy += amp * np.cos(arg) * k * math.sin(th[s])
    N = _normalize(np.stack([-dZx, -dZy, np.ones_like(X)]))
    return X, Y, Z, N


def heightfield_mirror(m=16, receiver_z=1.0, seed_offset=1):
    """Single-reflection heightfield: (m+1)^2 vertices on [-1,1]^2 (2 m^2
    triangles), z = 0.05 * sum of 4 seeded sinusoids (frequency 1-4, random
    direction and phase), interpolated analytic normals, a unit point light at
    (0,0,2) and a receiver plane z = receiver_z over [-2,2]^2.

    With the mirror facing +z and the light above it, reflected light travels
    upward, so the default receiver sits at z = +1 (between mirror and light);
    receiver_z = -1 gives the literal below-the-mirror plane, which receives
    almost nothing."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    X, Y, Z, N = _sinusoid_heightfield(m, -1.0, 1.0, 0.05, rng)
    pos, nrm = _grid_triangles(X, Y, Z, N)
    return _scene("R", pos, nrm, [0.0, 0.0, 2.0], [1.0],
                  [-2.0, -2.0, receiver_z], [4.0, 0.0, 0.0], [0.0, 4.0, 0.0],
                  name=f"heightfield{m}x{m}")


def _octahedral_sphere(levels):
    """Geodesic sphere from a subdivided octahedron: 8 * 4^levels triangles,
    vertices deduplicated across face seams, outward winding."""
    nseg = 2 ** levels
    corners = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    faces = []
    for sx in (0, 1):
        for sy in (2, 3):
            for sz in (4, 5):
                a, b, c = corners[sx], corners[sy], corners[sz]
                if np.dot(np.cross(b - a, c - a), a + b + c) < 0:
                    b, c = c, b
                faces.append((a, b, c))
    ii, jj = np.meshgrid(np.arange(nseg + 1), np.arange(nseg + 1), indexing="ij")
    keep = (ii + jj) <= nseg
    ii, jj = ii[keep], jj[keep]
    lid = -np.ones((nseg + 1, nseg + 1), dtype=np.int64)
    lid[ii, jj] = np.arange(ii.size)
    # local triangles on the (i, j) lattice
    up_i, up_j = np.meshgrid(np.arange(nseg), np.arange(nseg), indexing="ij")
    m_up = (up_i + up_j) <= nseg - 1
    m_dn = (up_i + up_j) <= nseg - 2
    ui, uj = up_i[m_up], up_j[m_up]
    di, dj = up_i[m_dn], up_j[m_dn]
    loc = np.concatenate([
        np.stack([lid[ui, uj], lid[ui + 1, uj], lid[ui, uj + 1]], 1),
        np.stack([lid[di + 1, dj], lid[di + 1, dj + 1], lid[di, dj + 1]], 1)])
    verts, tris = [], []
    for f, (a, b, c) in enumerate(faces):
        p = a[None] + (b - a)[None] * (ii[:, None] / nseg) + (c - a)[None] * (jj[:, None] / nseg)
        verts.append(p)
        tris.append(loc + f * ii.size)
    V = np.concatenate(verts)
    T = np.concatenate(tris)
    V = _normalize(V, axis=1)
    key = np.round(V * (1 << 20)).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    V = V[first]
    T = inv.reshape(-1)[T]
    return V, T


def _value_noise(P, cells_per_unit, rng, extent=1.25):
    """Trilinear interpolation of a seeded lattice of U[-1,1] values with the
    given number of lattice cells per unit length, evaluated at points P [k,3]."""
    n = int(math.ceil(2 * extent * cells_per_unit)) + 2
    lat = rng.uniform(-1.0, 1.0, (n, n, n))
    g = (P + extent) * cells_per_unit
    i0 = np.floor(g).astype(np.int64)
    t = g - i0
    out = np.zeros(P.shape[0])
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                w = (np.where(dx, t[:, 0], 1 - t[:, 0]) * np.where(dy, t[:, 1], 1 - t[:, 1])
                     * np.where(dz, t[:, 2], 1 - t[:, 2]))
                out += w * lat[i0[:, 0] + dx, i0[:, 1] + dy, i0[:, 2] + dz]
    return out


def displaced_sphere(levels=7, amp=0.02, seed_offset=2):
    """Single reflection off a displaced sphere: octahedral geodesic sphere with
    8*4^levels triangles (levels=7 gives 131072), radius 1 + amp * value noise
    (8 lattice cells per unit), area-weighted vertex normals; unit point light at
    (0,0,3); receiver plane z = -3 over [-5,5]^2 behind the sphere."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    V, T = _octahedral_sphere(levels)
    r = 1.0 + amp * _value_noise(V, 8.0, rng)
    V = V * r[:, None]
    p0, p1, p2 = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    fn = np.cross(p1 - p0, p2 - p0)  # |fn| = 2 * area, outward
    vn = np.zeros_like(V)
    for k in range(3):
        np.add.at(vn, T[:, k], fn)
    vn = _normalize(vn, axis=1)
    pos = np.concatenate([p0.T, p1.T, p2.T])
    nrm = np.concatenate([vn[T[:, 0]].T, vn[T[:, 1]].T, vn[T[:, 2]].T])
    return _scene("R", pos, nrm, [0.0, 0.0, 3.0], [1.0],
                  [-5.0, -5.0, -3.0], [10.0, 0.0, 0.0], [0.0, 10.0, 0.0],
                  name=f"sphere{len(T)}")


def water_surface(m=512, n_waves=32, n_lights=4, eta=1.0 / 1.5, seed_offset=3, amp=(0.01, 0.05),
                  wavelength=(0.05, 0.5), amp_scale=1.0, crop=None):
    """Single refraction through a water surface: (m+1)^2 vertices on [-1,1]^2
    (2 m^2 triangles), height = sum of n_waves seeded sine waves (amplitude and
    wavelength uniform in the given ranges, random direction and phase),
    analytic normals facing up (the incident side); n_lights unit point lights at
    xy ~ U[-1,1]^2, z ~ U[2,4]; receiver (pool floor) z = -1 over [-1,1]^2.
    crop = (i0, j0, k) keeps only the k x k cells from vertex (i0, j0) on: the
    same surface, lights and receiver at full resolution, 2 k^2 triangles."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    a = rng.uniform(amp[0], amp[1], n_waves) * amp_scale
    lam = rng.uniform(wavelength[0], wavelength[1], n_waves)
    th = rng.uniform(0, 2 * math.pi, n_waves)
    ph = rng.uniform(0, 2 * math.pi, n_waves)
    xs = np.linspace(-1.0, 1.0, m + 1)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    Z = np.zeros_like(X)
    dZx = np.zeros_like(X)
    dZy = np.zeros_like(X)
    for s in range(n_waves):
        k = 2 * math.pi / lam[s]
        arg = k * (X * math.cos(th[s]) + Y * math.sin(th[s])) + ph[s]
        Z += a[s] * np.sin(arg)
        dZx += a[s] * np.cos(arg) * k * math.cos(th[s])
        dZy += a[s] * np.cos(arg) * k * math.sin(th[s])
    N = _normalize(np.stack([-dZx, -dZy, np.ones_like(X)]))
    name = f"water{m}x{m}"
    if crop is not None:
        i0, j0, k = crop
        sl = (slice(i0, i0 + k + 1), slice(j0, j0 + k + 1))
        X, Y, Z, N = X[sl], Y[sl], Z[sl], N[(slice(None),) + sl]
        name += f"_crop{i0}_{j0}_{k}"
    pos, nrm = _grid_triangles(X, Y, Z, N)
    lx = rng.uniform(-1, 1, n_lights)
    ly = rng.uniform(-1, 1, n_lights)
    lz = rng.uniform(2, 4, n_lights)
    return _scene("T", pos, nrm, np.stack([lx, ly, lz]), np.ones(n_lights),
                  [-1.0, -1.0, -1.0], [2.0, 0.0, 0.0], [0.0, 2.0, 0.0], eta=eta,
                  name=name)


def facing_walls(m=64, amp=0.03, seed_offset=4):
    """Two specular vertices: wall A at x = -1 facing +x and wall B at x = +1
    facing -x, each an (m+1)^2-vertex heightfield over (y, z) in [-1,1] x [0,3]
    with 4 seeded sinusoid bumps of amplitude amp; unit point light at
    (0, 0, 2.5); receiver floor z = 0 over [-1,1]^2."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    walls = []
    for side in (-1.0, 1.0):
        ys = np.linspace(-1.0, 1.0, m + 1)
        zs = np.linspace(0.0, 3.0, m + 1)
        Yg, Zg = np.meshgrid(ys, zs, indexing="ij")
        f = rng.uniform(1.0, 4.0, 4)
        th = rng.uniform(0, 2 * math.pi, 4)
        ph = rng.uniform(0, 2 * math.pi, 4)
        H = np.zeros_like(Yg)
        dHy = np.zeros_like(Yg)
        dHz = np.zeros_like(Yg)
        for s in range(4):
            k = math.pi * f[s]
            arg = k * (Yg * math.cos(th[s]) + Zg * math.sin(th[s])) + ph[s]
            H += amp * np.sin(arg)
            dHy += amp * np.cos(arg) * k * math.cos(th[s])
            dHz += amp * np.cos(arg) * k * math.sin(th[s])
        # wall surface x = side * (1 - H) ... displaced toward the room interior by H
        X = side * (1.0 - H)
        # outward normal points into the room: -side * x-axis, tilted by the gradient
        Nx = -side * np.ones_like(Yg)
        Ny = -dHy * 1.0
        Nz = -dHz * 1.0
        # surface x = side*(1-H(y,z)); gradient of F = x - side*(1-H) is (1, side*dHy, side*dHz)
        Ny = -side * side * dHy  # == -dHy, written to keep the orientation explicit
        Nz = -side * side * dHz
        N = _normalize(np.stack([Nx, Ny * 1.0, Nz * 1.0]))
        # grid in (y, z): build triangles, then orient them to face the interior
        P = np.stack([X, Yg, Zg])
        pos, nrm = _grid_triangles(P[1], P[2], P[0], np.stack([N[1], N[2], N[0]]))
        # _grid_triangles took (y, z, x) as its (x, y, z); rotate the rows back
        pos = pos.reshape(3, 3, -1)[:, [2, 0, 1], :].reshape(9, -1)
        nrm = nrm.reshape(3, 3, -1)[:, [2, 0, 1], :].reshape(9, -1)
        e1 = pos[3:6] - pos[0:3]
        e2 = pos[6:9] - pos[0:3]
        gn = np.cross(e1.T, e2.T).T
        flip = np.sum(gn * (nrm[0:3] + nrm[3:6] + nrm[6:9]), axis=0) < 0
        pos[3:6, flip], pos[6:9, flip] = pos[6:9, flip].copy(), pos[3:6, flip].copy()
        nrm[3:6, flip], nrm[6:9, flip] = nrm[6:9, flip].copy(), nrm[3:6, flip].copy()
        walls.append((pos, nrm))
    (pa, na), (pb, nb) = walls
    return _scene("RR", pa, na, [0.0, 0.0, 2.5], [1.0],
                  [-1.0, -1.0, 0.0], [2.0, 0.0, 0.0], [0.0, 2.0, 0.0],
                  pos2=pb, nrm2=nb, name=f"walls{m}x{m}")


# --- tiny scenes for unit tests -------------------------------------------------

def double_mirror(light=(0.1, 0.2, 1.0), upper_z=2.0, receiver_z=1.5, half=1.5):
    """Two reflections between two parallel flat mirrors: mirror A (one large
    triangle in z = 0, facing up) and mirror B (one large triangle in
    z = upper_z, facing down); receiver z = receiver_z over [-half, half]^2.
    The light's image in A and then in B is a point source at
    (lx, ly, 2 upper_z + lz): the irradiance has a closed form."""
    b = 6.0  # each mirror is one triangle covering x, y >= -b, x + y <= 2b
    na = np.tile(np.array([0.0, 0.0, 1.0]), 3).reshape(9, 1)
    nb = np.tile(np.array([0.0, 0.0, -1.0]), 3).reshape(9, 1)
    pa = np.array([[-b, -b, 0.0], [3 * b, -b, 0.0], [-b, 3 * b, 0.0]]).reshape(9, 1)
    pb = np.array([[-b, -b, upper_z], [-b, 3 * b, upper_z], [3 * b, -b, upper_z]]).reshape(9, 1)
    return _scene("RR", pa, na, list(light), [1.0], [-half, -half, receiver_z], [2 * half, 0.0, 0.0],
                  [0.0, 2 * half, 0.0], pos2=pb, nrm2=nb, name="double_mirror")


def flat_mirror(light=(0.1, 0.2, 2.0), receiver_z=1.0, half=3.0):
    """One flat mirror triangle in z = 0 (constant normals), light above it and a
    receiver plane above the mirror.  The image-source construction gives the
    irradiance in closed form."""
    pos = np.array([-1, -1, 0, 1, -1, 0, -1, 1, 0], float).reshape(9, 1)
    nrm = np.array([0, 0, 1] * 3, float).reshape(9, 1)
    return _scene("R", pos, nrm, list(light), [1.0],
                  [-half, -half, receiver_z], [2 * half, 0, 0], [0, 2 * half, 0], name="flat_mirror")


def area_light(scene, a, b):
    """The scene with each point light replaced by a parallelogram light
    centred on it: corner epos - a/2 - b/2, edges a and b (the same for every
    emitter), stored as eedge [6][n_emit]."""
    s = dict(scene)
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    n = scene["epos"].shape[1]
    s["epos"] = _f32(scene["epos"].astype(np.float64) - 0.5 * (a + b)[:, None])
    s["eedge"] = _f32(np.concatenate([np.repeat(a[:, None], n, 1), np.repeat(b[:, None], n, 1)]))
    s["name"] = scene.get("name", "") + "_area"
    return s


def curved_triangles(n=4, seed=7, chain="R", eta=1.0, receiver_z=None):
    """n triangles in a row with seeded tilted vertex normals (a curved
    reflector or refractor).  Light above; receiver above (R) or below (T)."""
    rng = np.random.default_rng(SEED_BASE + 100 + seed)
    pos = np.zeros((9, n))
    nrm = np.zeros((9, n))
    for t in range(n):
        x0 = -1.0 + 2.0 * t / n
        w = 2.0 / n
        P = np.array([[x0, -0.6, 0.0], [x0 + w, -0.6, 0.02 * t], [x0 + 0.3 * w, 0.6, -0.01 * t]])
        if chain == "T":
            P[:, 2] = 0.0
        for k in range(3):
            nn = np.array([rng.uniform(-0.25, 0.25), rng.uniform(-0.25, 0.25), 1.0])
            pos[3 * k:3 * k + 3, t] = P[k]
            nrm[3 * k:3 * k + 3, t] = nn / np.linalg.norm(nn)
    if receiver_z is None:
        receiver_z = 1.0 if chain == "R" else -1.0
    half = 2.5
    return _scene(chain, pos, nrm, [0.05, -0.1, 2.0], [1.0],
                  [-half, -half, receiver_z], [2 * half, 0, 0], [0, 2 * half, 0], eta=eta,
                  name=f"curved{n}_{chain}")


# --- shading points ---------------------------------------------------------------

def receiver_points(scene, nu, nv=None, grid_res=512, cell_centre=True):
    """nu x nv shading points on the receiver, [3, nu*nv] float32, row-major in
    (u, v).  With cell_centre=True each point is moved to the centre of the
    bound-grid cell (grid_res^2 cells over [0,1]^2) that contains the regular
    (i+1/2)/nu sample, so no point lies on a cell edge."""
    nv = nu if nv is None else nv
    u = (np.arange(nu) + 0.5) / nu
    v = (np.arange(nv) + 0.5) / nv
    if cell_centre:
        u = (np.floor(u * grid_res) + 0.5) / grid_res
        v = (np.floor(v * grid_res) + 0.5) / grid_res
    U, Vv = np.meshgrid(u, v, indexing="ij")
    q0 = scene["q0"].astype(np.float64)
    f1 = scene["f1"].astype(np.float64)
    f2 = scene["f2"].astype(np.float64)
    P = q0[:, None] + f1[:, None] * U.reshape(1, -1) + f2[:, None] * Vv.reshape(1, -1)
    return _f32(P)


def random_points(scene, n, seed=0, grid_res=512):
    """n seeded shading points at random bound-grid cell centres of the receiver."""
    rng = np.random.default_rng(SEED_BASE + 1000 + seed)
    cu = rng.integers(0, grid_res, n)
    cv = rng.integers(0, grid_res, n)
    u = (cu + 0.5) / grid_res
    v = (cv + 0.5) / grid_res
    q0 = scene["q0"].astype(np.float64)
    f1 = scene["f1"].astype(np.float64)
    f2 = scene["f2"].astype(np.float64)
    P = q0[:, None] + f1[:, None] * u[None] + f2[:, None] * v[None]
    return _f32(P)


def config_scene(index):
    """Scene of workload `index` (1-4) at full size."""
    if index == 1:
        return heightfield_mirror(16)
    if index == 2:
        return displaced_sphere(7)
    if index == 3:
        return water_surface(512)
    if index == 4:
        return facing_walls(64)
    raise ValueError(index)
