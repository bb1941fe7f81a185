"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This module holds no DG arithmetic: it samples analytic initial conditions
(stated in primitive variables, converted to conserved variables by the
ideal-gas relation that defines the state) at the nodal positions of a
periodic Cartesian mesh.  The positions come from numpy's library
Gauss-Legendre rule; both solvers compute their own quadrature.

Array layout of every state: Q[f, ez, ey, ex, k, j, i], fields
f = (rho, rho u, rho v, rho w, rho E), element index ex fastest among
elements, node index i (x direction) fastest inside an element.

Workloads (all periodic, gamma = 1.4 unless stated):
  density_wave  -- rho = 1 + A sin(2 pi k.(x - u t)), u, pressure uniform.
                   An exact solution of the Euler equations (pure advection).
  tgv           -- Taylor-Green vortex on [0, 2 pi]^3 at Mach M:
                   u = V0 sin x cos y cos z, v = -V0 cos x sin y cos z, w = 0,
                   p = p0 + rho0 V0^2/16 (cos 2x + cos 2y)(cos 2z + 2),
                   p0 = rho0 V0^2 / (gamma M^2), rho = rho0 p / p0.
  perturbed_tgv -- tgv plus seeded smooth sine perturbations of every
                   primitive variable (adjoint workload).
  random_smooth -- seeded smooth random state with O(1) variation (parity).
  batch_specs   -- seeded list of independent instances (kind, n, p, ...).
"""

import math

import numpy as np

GAMMA = 1.4
FIELDS = ("rho", "rho_u", "rho_v", "rho_w", "rho_E")


def _gl_nodes(p):
    x, _ = np.polynomial.legendre.leggauss(p + 1)
    return x


def node_coords(n, p, L):
    """Physical node coordinates X, Y, Z, each shaped [nz, ny, nx, N, N, N]
    (element (ex, ey, ez) covers [ex h_x, (ex+1) h_x] etc.)."""
    nx, ny, nz = n
    Lx, Ly, Lz = L
    xi = _gl_nodes(p)
    N = p + 1
    hx, hy, hz = Lx / nx, Ly / ny, Lz / nz
    ex = np.arange(nx)[None, None, :, None, None, None]
    ey = np.arange(ny)[None, :, None, None, None, None]
    ez = np.arange(nz)[:, None, None, None, None, None]
    ri = xi[None, None, None, None, None, :]
    rj = xi[None, None, None, None, :, None]
    rk = xi[None, None, None, :, None, None]
    shape = (nz, ny, nx, N, N, N)
    X = np.broadcast_to(ex * hx + (ri + 1.0) * (hx / 2.0), shape)
    Y = np.broadcast_to(ey * hy + (rj + 1.0) * (hy / 2.0), shape)
    Z = np.broadcast_to(ez * hz + (rk + 1.0) * (hz / 2.0), shape)
    return X, Y, Z


def conserved(rho, u, v, w, pres, gamma=GAMMA):
    """Conserved state from primitive fields (the ideal-gas state relation)."""
    en = pres / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    out = np.stack(np.broadcast_arrays(rho, rho * u, rho * v, rho * w, en))
    return np.ascontiguousarray(out, dtype=np.float64)


def _mesh(n):
    if np.isscalar(n):
        return (int(n),) * 3
    return tuple(int(v) for v in n)


def density_wave(n, p, amp=0.2, k=(1, 1, 1), vel=(1.0, 1.0, 1.0), pres=1.0,
                 t=0.0, L=(1.0, 1.0, 1.0), gamma=GAMMA):
    """rho = 1 + amp sin(2 pi k.(x - vel t)), velocity ``vel``, pressure
    ``pres``, on [0,Lx]x[0,Ly]x[0,Lz]."""
    n = _mesh(n)
    X, Y, Z = node_coords(n, p, L)
    ph = 2.0 * math.pi * (k[0] * (X - vel[0] * t) + k[1] * (Y - vel[1] * t)
                          + k[2] * (Z - vel[2] * t))
    rho = 1.0 + amp * np.sin(ph)
    one = np.ones_like(rho)
    return conserved(rho, vel[0] * one, vel[1] * one, vel[2] * one, pres * one, gamma)


def density_wave_exact(X, Y, Z, t, amp=0.2, k=(1, 1, 1), vel=(1.0, 1.0, 1.0)):
    """Exact density of the advected wave at arbitrary points and time t."""
    ph = 2.0 * math.pi * (k[0] * (X - vel[0] * t) + k[1] * (Y - vel[1] * t)
                          + k[2] * (Z - vel[2] * t))
    return 1.0 + amp * np.sin(ph)


def tgv_primitives(X, Y, Z, mach=0.1, V0=1.0, rho0=1.0, gamma=GAMMA,
                   rho_const=False, mult=1):
    """Primitive Taylor-Green fields (rho, u, v, w, p) at points."""
    x, y, z = mult * X, mult * Y, mult * Z
    p0 = rho0 * V0 * V0 / (gamma * mach * mach)
    u = V0 * np.sin(x) * np.cos(y) * np.cos(z)
    v = -V0 * np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(u)
    pres = p0 + rho0 * V0 * V0 / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    rho = np.full_like(u, rho0) if rho_const else rho0 * pres / p0
    return rho, u, v, w, pres


def tgv(n, p, mach=0.1, V0=1.0, rho0=1.0, gamma=GAMMA, rho_const=False, mult=1,
        L=(2 * math.pi,) * 3):
    """Taylor-Green vortex on [0, 2 pi]^3 (see module docstring)."""
    n = _mesh(n)
    X, Y, Z = node_coords(n, p, L)
    rho, u, v, w, pres = tgv_primitives(X, Y, Z, mach, V0, rho0, gamma, rho_const, mult)
    return conserved(rho, u, v, w, pres, gamma)


def _smooth_field(rng, X, Y, Z, L, kmax, amp):
    """sum over |k|_inf <= kmax of a_k sin(2 pi k.x/L + phi_k), normalised
    so that its maximum magnitude at the nodes is ``amp``."""
    f = np.zeros(X.shape)
    for kx in range(-kmax, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            for kz in range(-kmax, kmax + 1):
                if kx == 0 and ky == 0 and kz == 0:
                    continue
                a = rng.standard_normal()
                ph = rng.uniform(0.0, 2.0 * math.pi)
                f += a * np.sin(2 * math.pi * (kx * X / L[0] + ky * Y / L[1] + kz * Z / L[2]) + ph)
    m = np.max(np.abs(f))
    return f * (amp / m) if m > 0 else f


def perturbed_tgv(n, p, seed=1, amp=1e-2, kmax=2, mach=0.1, V0=1.0, rho0=1.0,
                  gamma=GAMMA, L=(2 * math.pi,) * 3):
    """TGV base state with seeded smooth perturbations: rho and p are
    multiplied by (1 + f), f of max amplitude ``amp``; each velocity gets
    V0 * g added, g of max amplitude ``amp``."""
    n = _mesh(n)
    rng = np.random.default_rng(seed)
    X, Y, Z = node_coords(n, p, L)
    rho, u, v, w, pres = tgv_primitives(X, Y, Z, mach, V0, rho0, gamma)
    rho = rho * (1.0 + _smooth_field(rng, X, Y, Z, L, kmax, amp))
    u = u + V0 * _smooth_field(rng, X, Y, Z, L, kmax, amp)
    v = v + V0 * _smooth_field(rng, X, Y, Z, L, kmax, amp)
    w = w + V0 * _smooth_field(rng, X, Y, Z, L, kmax, amp)
    pres = pres * (1.0 + _smooth_field(rng, X, Y, Z, L, kmax, amp))
    return conserved(rho, u, v, w, pres, gamma)


def random_smooth(n, p, seed=0, L=(1.0, 1.0, 1.0), noise=0.0, gamma=GAMMA, mach=0.5):
    """Seeded smooth random state with O(1) variation in every primitive
    (rho in [0.6, 1.4], |u| up to about ``mach`` times the sound speed), plus
    optional node-wise uniform noise of relative size ``noise`` (makes the
    state discontinuous between elements, exercising the face flux)."""
    n = _mesh(n)
    rng = np.random.default_rng(seed)
    X, Y, Z = node_coords(n, p, L)
    rho = 1.0 + _smooth_field(rng, X, Y, Z, L, 1, 0.4)
    pres = 1.0 + _smooth_field(rng, X, Y, Z, L, 1, 0.4)
    c = math.sqrt(gamma)
    u = _smooth_field(rng, X, Y, Z, L, 1, mach * c)
    v = _smooth_field(rng, X, Y, Z, L, 1, mach * c)
    w = _smooth_field(rng, X, Y, Z, L, 1, mach * c)
    if noise > 0:
        sh = rho.shape
        rho = rho * (1.0 + noise * rng.uniform(-1, 1, sh))
        pres = pres * (1.0 + noise * rng.uniform(-1, 1, sh))
        u = u + noise * rng.uniform(-1, 1, sh)
        v = v + noise * rng.uniform(-1, 1, sh)
        w = w + noise * rng.uniform(-1, 1, sh)
    return conserved(rho, u, v, w, pres, gamma)


def uniform_state(n, p, rho, vel, pres, gamma=GAMMA):
    """A uniform (free-stream) state."""
    n = _mesh(n)
    N = p + 1
    shape = (n[2], n[1], n[0], N, N, N)
    one = np.ones(shape)
    return conserved(rho * one, vel[0] * one, vel[1] * one, vel[2] * one, pres * one, gamma)


def gaussian_directions(Q, count, seed0=1000):
    """``count`` seeded Gaussian directions per unknown, each field scaled by
    that field's RMS, every direction normalised to unit l2 norm."""
    rms = np.sqrt(np.mean(Q.reshape(Q.shape[0], -1) ** 2, axis=1))
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        d = rng.standard_normal(Q.shape) * rms.reshape((-1,) + (1,) * (Q.ndim - 1))
        out.append(d / np.linalg.norm(d))
    return out


def batch_specs(count=512, seed=15698, nmin=6, nmax=24, pmin=1, pmax=5):
    """Seeded independent instances: kind ~ Bernoulli(1/2) between a density
    wave on [0,1]^3 (random k in {-2..2}^3 minus 0) and a TGV on [0,2pi]^3
    (wave multiplier in {1,2}, V0 = A, Mach 0.1); n ~ U{nmin..nmax} per
    instance (n^3 elements); p ~ U{pmin..pmax}; A ~ U[0.05, 0.3]."""
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(count):
        kind = "wave" if rng.integers(0, 2) == 0 else "tgv"
        n = int(rng.integers(nmin, nmax + 1))
        p = int(rng.integers(pmin, pmax + 1))
        amp = float(rng.uniform(0.05, 0.3))
        if kind == "wave":
            while True:
                k = tuple(int(v) for v in rng.integers(-2, 3, size=3))
                if k != (0, 0, 0):
                    break
            specs.append(dict(kind=kind, n=n, p=p, amp=amp, k=k, mult=1,
                              L=(1.0, 1.0, 1.0)))
        else:
            mult = int(rng.integers(1, 3))
            specs.append(dict(kind=kind, n=n, p=p, amp=amp, k=None, mult=mult,
                              L=(2 * math.pi,) * 3))
    return specs


def batch_state(spec, gamma=GAMMA):
    """Initial state of one ``batch_specs`` entry."""
    if spec["kind"] == "wave":
        return density_wave(spec["n"], spec["p"], amp=spec["amp"], k=spec["k"],
                            L=spec["L"], gamma=gamma)
    return tgv(spec["n"], spec["p"], mach=0.1, V0=spec["amp"], mult=spec["mult"],
               L=spec["L"], gamma=gamma)


def varp_coords(n, degrees, L=(1.0, 1.0, 1.0)):
    """Node coordinates of a periodic mesh with a degree per element
    (degrees[ez, ey, ex]): a list, element order e = (ez ny + ey) nx + ex,
    of (X, Y, Z) arrays shaped [N_e, N_e, N_e] (k, j, i; i fastest)."""
    nx, ny, nz = _mesh(n)
    deg = np.asarray(degrees, dtype=int).reshape(nz, ny, nx)
    h = (L[0] / nx, L[1] / ny, L[2] / nz)
    out = []
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                xi = _gl_nodes(int(deg[ez, ey, ex]))
                K, J, I = np.meshgrid(xi, xi, xi, indexing="ij")
                out.append((ex * h[0] + (I + 1.0) * (h[0] / 2.0), ey * h[1] + (J + 1.0) * (h[1] / 2.0),
                            ez * h[2] + (K + 1.0) * (h[2] / 2.0)))
    return out


def varp_offsets(degrees):
    """First node of every element (and the total), element order."""
    n3 = (np.asarray(degrees, dtype=np.int64).reshape(-1) + 1) ** 3
    return np.concatenate([[0], np.cumsum(n3)])


def varp_state(n, degrees, primitive, L=(1.0, 1.0, 1.0), gamma=GAMMA):
    """State [5, total nodes] of a variable-degree mesh from a function
    primitive(X, Y, Z) -> (rho, u, v, w, p), element blocks back to back
    (evaluated degree by degree, all elements of a degree at once)."""
    nx, ny, nz = _mesh(n)
    deg = np.asarray(degrees, dtype=np.int64).reshape(-1)
    if deg.size != nx * ny * nz:
        raise ValueError("one degree per element")
    h = (L[0] / nx, L[1] / ny, L[2] / nz)
    off = varp_offsets(deg)
    out = np.empty((5, int(off[-1])))
    e_all = np.arange(deg.size)
    for p in np.unique(deg):
        es = e_all[deg == p]
        N = int(p) + 1
        xi = _gl_nodes(int(p))
        ex, ey, ez = es % nx, (es // nx) % ny, es // (nx * ny)
        K, J, I = np.meshgrid(xi, xi, xi, indexing="ij")
        X = ex[:, None, None, None] * h[0] + (I[None] + 1.0) * (h[0] / 2.0)
        Y = ey[:, None, None, None] * h[1] + (J[None] + 1.0) * (h[1] / 2.0)
        Z = ez[:, None, None, None] * h[2] + (K[None] + 1.0) * (h[2] / 2.0)
        q = conserved(*primitive(X, Y, Z), gamma=gamma).reshape(5, len(es), N ** 3)
        idx = off[es][:, None] + np.arange(N ** 3)[None, :]
        out[:, idx] = q
    return out


def random_degrees(n, pmin, pmax, seed):
    """Seeded degree per element, uniform in pmin..pmax, shaped [nz, ny, nx]."""
    nx, ny, nz = _mesh(n)
    return np.random.default_rng(seed).integers(pmin, pmax + 1, size=(nz, ny, nx))


def tgv_indicator(n, L=(2 * np.pi, 2 * np.pi, 2 * np.pi)):
    """The Taylor-Green vortex's initial enstrophy density at the cell
    centres [nz, ny, nx], as an hp indicator would read it: s = |curl u| / 2
    in [0, 1] (V0 = 1)."""
    nx, ny, nz = _mesh(n)
    x = (np.arange(nx) + 0.5) * (L[0] / nx)
    y = (np.arange(ny) + 0.5) * (L[1] / ny)
    z = (np.arange(nz) + 0.5) * (L[2] / nz)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    w1 = -np.cos(X) * np.sin(Y) * np.sin(Z)
    w2 = -np.sin(X) * np.cos(Y) * np.sin(Z)
    w3 = 2 * np.sin(X) * np.sin(Y) * np.cos(Z)
    return np.sqrt(w1 ** 2 + w2 ** 2 + w3 ** 2) / 2.0


def tgv_degrees(n, pmin=3, pmax=5, L=(2 * np.pi, 2 * np.pi, 2 * np.pi)):
    """Degree per element [nz, ny, nx] driven by the Taylor-Green vortex's
    initial enstrophy density at the element centre (``tgv_indicator``):
    degree pmin + round((pmax - pmin) s).  On 48^3 with 3..5: 22% / 72% / 5%
    of the elements, 6% of the faces between two degrees."""
    s = tgv_indicator(n, L)
    return (pmin + np.rint((pmax - pmin) * s)).astype(np.int64)


def tgv_refined_mesh(n, threshold=0.7, pmin=3, pmax=5, L=(2 * np.pi, 2 * np.pi, 2 * np.pi)):
    """An hp mesh of the Taylor-Green vortex: the cells whose enstrophy
    indicator is at least ``threshold`` refined once, every cell's degree
    from ``tgv_degrees`` (a refined cell's eight children take its degree).
    Returns (refine [nz, ny, nx], degrees per element in element order).  On
    40^3 with 0.7: 7.8% of the cells refined, 98944 elements, 14.0 M nodes,
    16896 hanging sub-faces."""
    refine = (tgv_indicator(n, L) >= threshold).astype(np.int64)
    cdeg = tgv_degrees(n, pmin, pmax, L)
    return refine, np.repeat(cdeg.reshape(-1), np.where(refine.reshape(-1) == 1, 8, 1))


def hp_geometry(n, refine, L):
    """Origins [E, 3], sizes [E, 3] and levels [E] of the elements of a
    refined mesh, in element order (as ``hp_elements``)."""
    nx, ny, nz = _mesh(n)
    ref = np.asarray(refine, dtype=np.int64).reshape(-1)
    if ref.size != nx * ny * nz:
        raise ValueError(f"{ref.size} refinement flags for {nx * ny * nz} cells")
    h = np.array([L[0] / nx, L[1] / ny, L[2] / nz])
    c = np.arange(nx * ny * nz)
    base = np.stack([c % nx, (c // nx) % ny, c // (nx * ny)], axis=1) * h
    count = np.where(ref == 1, 8, 1)
    cell = np.repeat(c, count)
    # rank of each element inside its cell: the child index (kz, ky, kx)
    rank = np.arange(cell.size) - np.repeat(np.cumsum(count) - count, count)
    lev = ref[cell]
    kid = np.stack([rank % 2, (rank // 2) % 2, rank // 4], axis=1)
    size = h[None, :] / np.where(lev == 1, 2.0, 1.0)[:, None]
    x0 = base[cell] + kid * size
    return x0, size, lev


def hp_elements(n, refine, L=(1.0, 1.0, 1.0)):
    """Elements of a periodic base mesh whose cells refine[cz, cy, cx] = 1 are
    split once into 2 x 2 x 2 children: a list, in element order (cells
    c = (cz ny + cy) nx + cx ascending, a refined cell's children (kz, ky, kx)
    with kx fastest), of (origin [3], size [3], level)."""
    x0, size, lev = hp_geometry(n, refine, L)
    return [(x0[e], size[e], int(lev[e])) for e in range(len(lev))]


def hp_state(n, refine, degrees, primitive, L=(1.0, 1.0, 1.0), gamma=GAMMA):
    """State [5, total nodes] of a refined mesh (hp_elements) with one degree
    per element (element order) from primitive(X, Y, Z) -> (rho, u, v, w, p),
    evaluated per degree for all elements of that degree at once."""
    x0, size, _ = hp_geometry(n, refine, L)
    deg = np.asarray(degrees, dtype=np.int64).reshape(-1)
    if deg.size != x0.shape[0]:
        raise ValueError(f"{deg.size} degrees for {x0.shape[0]} elements")
    off = varp_offsets(deg)
    out = np.empty((5, int(off[-1])))
    for p in np.unique(deg):
        es = np.flatnonzero(deg == p)
        xi = _gl_nodes(int(p))
        K, J, I = (a.reshape(-1) for a in np.meshgrid(xi, xi, xi, indexing="ij"))
        X = x0[es, 0, None] + (I[None, :] + 1.0) * (size[es, 0, None] / 2.0)
        Y = x0[es, 1, None] + (J[None, :] + 1.0) * (size[es, 1, None] / 2.0)
        Z = x0[es, 2, None] + (K[None, :] + 1.0) * (size[es, 2, None] / 2.0)
        q = conserved(*primitive(X, Y, Z), gamma=gamma)
        idx = off[es, None] + np.arange(I.size)[None, :]
        for f in range(5):
            out[f, idx] = np.broadcast_to(q[f], X.shape)
    return out


def random_refinement(n, fraction, seed):
    """Seeded refine[cz, cy, cx]: each cell refined with the given probability."""
    nx, ny, nz = _mesh(n)
    return (np.random.default_rng(seed).random((nz, ny, nx)) < fraction).astype(np.int64)
