"""Seeded synthetic inputs for the DG right-hand-side path.

This module produces *inputs only*: periodic tetrahedral box meshes (vertex
coordinates and global vertex ids) and initial states evaluated at caller-given
node coordinates.  It contains none of the discretisation's arithmetic (no node
sets, operators, geometric factors, fluxes or time stepping), so that the CPU
oracle and the GPU library can both be fed from it without sharing any of the
method.

Workloads (the paper's periodic isentropic-vortex Euler benchmark, Sec. 5.2,
stands in for by these synthetic meshes and states):

* box [0, L]^3 split into n^3 cubes, each cut into 6 Kuhn tetrahedra along the
  main diagonal; vertices jittered per unique periodic vertex by U[-a h, a h]
  per component (h = L/n), which keeps the mesh periodic and its volume L^3;
* isentropic vortex (strength beta, free-stream Mach 0.5 along +x, column along
  z) on an ideal gas, optionally with a smooth periodic entropy perturbation of
  the density;
* constant states and "entropy waves" (constant velocity and pressure,
  arbitrary density) used by invariance tests;
* periodic rectilinear boxes of hexahedra (jittered grid lines) for the
  tensor-product elements of the paper's own benchmarks (Sec. 5.2).
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 1.4

# Kuhn (Freudenthal) subdivision: one tetrahedron per permutation of the axes,
# walking from the cube's lower corner to its upper corner.
_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))
_PERM_SIGN = (1, -1, -1, 1, 1, -1)


def kuhn_mesh(dims, lengths, jitter: float = 0.05, seed: int = 0):
    """Periodic box mesh of nx*ny*nz cubes (cells) x 6 tets.

    dims = (nx, ny, nz) cells, lengths = (Lx, Ly, Lz).  Returns
    ``(elem_xyz, elem_vid)``:
      elem_xyz  float64 [E, 4, 3]  unwrapped vertex coordinates (positive volume)
      elem_vid  int64   [E, 4]     global vertex ids; periodic images share ids
    Element id = 6 * (i + nx * (j + ny * k)) + perm, perm in the order
    xyz, xzy, yxz, yzx, zxy, zyx.  Tets of odd permutations swap their last two
    vertices so every element is positively oriented.  Each unique periodic
    vertex is moved by U[-jitter h_d, jitter h_d] in each component d.
    """
    nx, ny, nz = (int(v) for v in dims)
    if min(nx, ny, nz) < 1:
        raise ValueError("cell counts must be >= 1")
    h = np.array([lengths[0] / nx, lengths[1] / ny, lengths[2] / nz])
    rng = np.random.default_rng(seed)
    jit = rng.uniform(-1.0, 1.0, size=(nx * ny * nz, 3)) * (jitter * h)[None, :]

    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ijk = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)  # cell c = i + nx*(j + ny*k)
    E = 6 * nx * ny * nz
    elem_lat = np.zeros((E, 4, 3), dtype=np.int64)
    for pi, perm in enumerate(_PERMS):
        p0 = ijk.copy()
        p1 = p0.copy()
        p1[:, perm[0]] += 1
        p2 = p1.copy()
        p2[:, perm[1]] += 1
        p3 = p2.copy()
        p3[:, perm[2]] += 1
        verts = (p0, p1, p2, p3) if _PERM_SIGN[pi] > 0 else (p0, p1, p3, p2)
        for v in range(4):
            elem_lat[pi::6, v, :] = verts[v]
    wrapped = elem_lat % np.array([nx, ny, nz])
    elem_vid = wrapped[..., 0] + nx * (wrapped[..., 1] + ny * wrapped[..., 2])
    elem_xyz = elem_lat.astype(np.float64) * h[None, None, :] + jit[elem_vid]
    return elem_xyz, elem_vid.astype(np.int64)


def kuhn_box_mesh(n: int, L: float = 10.0, jitter: float = 0.05, seed: int = 0):
    """Cubic periodic box [0, L]^3 of n^3 cubes x 6 tets (see kuhn_mesh)."""
    return kuhn_mesh((n, n, n), (L, L, L), jitter, seed)


def rectilinear_grid(dims, lengths, jitter: float = 0.05, seed: int = 0):
    """Grid lines of a periodic rectilinear box of nx * ny * nz hexahedra.

    Returns three arrays g_d of n_d + 1 strictly increasing coordinates: line
    i of axis d sits at i h_d + U[-jitter h_d, jitter h_d] (h_d = L_d / n_d)
    for i < n_d, and the last line is the first one shifted by the period,
    g_d[n_d] = g_d[0] + L_d, so the box stays periodic with volume L^3 and
    every cell is an axis-aligned box (an affine element).  Cell (i, j, k)
    spans [g_x[i], g_x[i+1]] x [g_y[j], g_y[j+1]] x [g_z[k], g_z[k+1]]."""
    if not 0.0 <= jitter < 0.5:
        raise ValueError("jitter must be in [0, 0.5)")
    rng = np.random.default_rng(seed)
    out = []
    for n, L in zip(dims, lengths):
        n = int(n)
        if n < 1:
            raise ValueError("cell counts must be >= 1")
        h = L / n
        g = np.arange(n + 1) * h
        g[:n] += rng.uniform(-jitter * h, jitter * h, n)
        g[n] = g[0] + L
        out.append(g)
    return tuple(out)


def rectilinear_box(n: int, L: float = 10.0, jitter: float = 0.05, seed: int = 0):
    """Cubic periodic rectilinear box of n^3 hexahedra (see rectilinear_grid)."""
    return rectilinear_grid((n, n, n), (L, L, L), jitter, seed)


def vortex_slab_mesh(n: int, L: float = 10.0, nz: int = 3, jitter: float = 0.05, seed: int = 0):
    """n x n x nz cubes of side L/n: a thin periodic slab for the z-independent
    vortex, so that in-plane resolution can be raised cheaply."""
    h = L / n
    return kuhn_mesh((n, n, nz), (L, L, nz * h), jitter, seed)


def _wrap(d, L):
    return (d + 0.5 * L) % L - 0.5 * L


def primitive_to_conserved(rho, u, v, w, p, gamma=GAMMA):
    """Ideal-gas conserved variables (rho, rho u, rho v, rho w, E)."""
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E])


def vortex_primitive(xyz, t=0.0, beta=5.0, center=(5.0, 5.0), mach=0.5, L=10.0, gamma=GAMMA, radius=1.0):
    """Isentropic vortex (Shu 1998; Yee, Sandham & Djomehri 1999) in a periodic box.

    rho_inf = p_inf = 1, free stream u_inf = mach * sqrt(gamma) along +x, column
    along z, core radius ``radius`` (distances scaled by 1/radius).  The exact
    solution at time t is the t = 0 field translated by u_inf * t (periodic
    wrap, nearest image).  Returns (rho, u, v, w, p) arrays
    shaped like ``xyz[..., 0]``.
    """
    uinf = mach * math.sqrt(gamma)
    x = xyz[..., 0]
    y = xyz[..., 1]
    dx = _wrap(x - (center[0] + uinf * t), L) / radius
    dy = _wrap(y - center[1], L) / radius
    r2 = dx * dx + dy * dy
    ex = np.exp(0.5 * (1.0 - r2))
    u = uinf - beta / (2.0 * math.pi) * dy * ex
    v = beta / (2.0 * math.pi) * dx * ex
    w = np.zeros_like(x)
    T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi * math.pi) * ex * ex
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    return rho, u, v, w, p


def density_perturbation(seed: int, modes: int = 4, amplitude: float = 1e-2, kmax: int = 4):
    """Seeded smooth periodic perturbation parameters: integer wave vectors in
    {1..kmax}^3, non-negative weights summing to one, phases in [0, 2 pi)."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, kmax + 1, size=(modes, 3))
    a = rng.uniform(0.0, 1.0, size=modes)
    a = a / a.sum()
    phi = rng.uniform(0.0, 2.0 * math.pi, size=modes)
    return {"k": k, "a": a, "phi": phi, "amplitude": amplitude}


def apply_density_perturbation(rho, xyz, pert, L=10.0):
    s = np.zeros_like(rho)
    for m in range(len(pert["a"])):
        arg = 2.0 * math.pi * (xyz @ pert["k"][m].astype(np.float64)) / L + pert["phi"][m]
        s = s + pert["a"][m] * np.sin(arg)
    return rho * (1.0 + pert["amplitude"] * s)


def vortex_state(xyz, t=0.0, beta=5.0, center=(5.0, 5.0), L=10.0, pert=None, gamma=GAMMA, radius=1.0):
    """Conserved state q[5][E][Np] of the (optionally perturbed) vortex at the
    given node coordinates ``xyz[E][Np][3]``."""
    rho, u, v, w, p = vortex_primitive(xyz, t=t, beta=beta, center=center, L=L, gamma=gamma, radius=radius)
    if pert is not None:
        rho = apply_density_perturbation(rho, xyz, pert, L=L)
    return np.ascontiguousarray(primitive_to_conserved(rho, u, v, w, p, gamma))


def constant_state(shape, rho=1.3, vel=(0.3, -0.2, 0.1), p=0.9, gamma=GAMMA):
    one = np.ones(shape)
    return np.ascontiguousarray(
        primitive_to_conserved(rho * one, vel[0] * one, vel[1] * one, vel[2] * one, p * one, gamma))


def entropy_wave_state(xyz, rho_fn, vel=(0.4, -0.25, 0.15), p=1.0, gamma=GAMMA):
    """Constant velocity and pressure with density rho_fn(xyz)."""
    rho = rho_fn(xyz)
    one = np.ones_like(rho)
    return np.ascontiguousarray(
        primitive_to_conserved(rho, vel[0] * one, vel[1] * one, vel[2] * one, p * one, gamma))


# Named workloads (mesh seed, perturbation seed) used by the tests and the bench.
WORKLOADS = {
    "vortex_p2_4cubed": dict(n=4, order=2, jitter=0.05, mesh_seed=1001, pert_seed=None),
    "vortex_pert_p3_48cubed": dict(n=48, order=3, jitter=0.03, mesh_seed=1002, pert_seed=2002),
}



def batch_specs(n_meshes: int = 64, n_min: int = 4, n_max: int = 40, seed: int = 5001, mesh_seed0: int = 5100):
    """Seeded specification of a batch of independent periodic vortex boxes
    [0, 10]^3: box size n ~ U{n_min..n_max} cubes per side (6 n^3 tets),
    order p ~ U{1..4}, vortex centre ~ U[3, 7]^2, strength beta ~ U[3, 5],
    5 % vertex jitter; mesh i has seed mesh_seed0 + i."""
    rng = np.random.default_rng(seed)
    n = rng.integers(n_min, n_max + 1, n_meshes)
    p = rng.integers(1, 5, n_meshes)
    centre = rng.uniform(3.0, 7.0, (n_meshes, 2))
    beta = rng.uniform(3.0, 5.0, n_meshes)
    return [dict(n=int(n[i]), order=int(p[i]), jitter=0.05, mesh_seed=mesh_seed0 + i,
                 center=(float(centre[i, 0]), float(centre[i, 1])), beta=float(beta[i]))
            for i in range(n_meshes)]

# ---------------------------------------------------------------------------
# Reacting-flow inputs: seeded synthetic species data, mechanism and fields.
# These are input tables only (the thermodynamic and kinetic laws that use
# them live in the library and, separately, in the oracle).

R_UNIVERSAL = 8.314462618  # J / (mol K)
N_SPECIES = 7
N_REACTIONS = 3
# R1: S1 + S2 -> S3 + S4 ;  R2: S3 + S2 -> S5 ;  R3: S4 + S5 -> S6 ;  S7 inert
NU_REACTANTS = np.array([[1, 1, 0, 0, 0, 0, 0], [0, 1, 1, 0, 0, 0, 0], [0, 0, 0, 1, 1, 0, 0]], dtype=np.float64)
NU_PRODUCTS = np.array([[0, 0, 1, 1, 0, 0, 0], [0, 0, 0, 0, 1, 0, 0], [0, 0, 0, 0, 0, 1, 0]], dtype=np.float64)


def synthetic_thermo(seed: int = 3003):
    """Seeded 7-species table: molar masses W [kg/mol] that balance the three
    reactions' mass, and single-range polynomial coefficients a[k] = (a1..a6)
    with cp_k / R_k = a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4 in [2.5, 10] and
    increasing on [200, 4000] K, and a6 [K] set from seeded molar formation
    enthalpies at 298.15 K so that every reaction is exothermic."""
    rng = np.random.default_rng(seed)
    W = np.zeros(N_SPECIES)
    W[0] = rng.uniform(0.010, 0.020)
    W[1] = rng.uniform(0.025, 0.035)
    W[2] = rng.uniform(0.010, W[0] + W[1] - 0.008)
    W[3] = W[0] + W[1] - W[2]
    W[4] = W[2] + W[1]
    W[5] = W[3] + W[4]
    W[6] = rng.uniform(0.026, 0.030)
    a = np.zeros((N_SPECIES, 6))
    for k in range(N_SPECIES):
        c = np.array([rng.uniform(2.5, 3.5), rng.uniform(0.5, 2.5), rng.uniform(0.0, 2.0),
                      rng.uniform(0.0, 1.0), rng.uniform(0.0, 0.5)])
        # cp/R = sum_m c_m s^m with s = (T - 200) / 3800: expand in powers of T
        poly = np.zeros(5)
        for m in range(5):
            # (T - 200)^m / 3800^m = sum_j binom(m, j) T^j (-200)^(m-j) / 3800^m
            for j in range(m + 1):
                poly[j] += c[m] * math.comb(m, j) * (-200.0) ** (m - j) / 3800.0 ** m
        a[k, :5] = poly
    h_form = np.array([50e3, 0.0, -100e3, -150e3, -250e3, -500e3, 0.0]) * rng.uniform(0.9, 1.1, N_SPECIES)
    T0 = 298.15
    for k in range(N_SPECIES):
        p5 = a[k, 0] * T0 + a[k, 1] * T0 ** 2 / 2 + a[k, 2] * T0 ** 3 / 3 + a[k, 3] * T0 ** 4 / 4 + a[k, 4] * T0 ** 5 / 5
        a[k, 5] = h_form[k] / R_UNIVERSAL - p5
    return {"W": W, "a": a}


def synthetic_mechanism(seed: int = 3004):
    """Seeded irreversible 3-step mechanism: pre-exponential factors A
    log-uniform in [1e8, 1e12] (SI, mol-m^3-s), activation energies Ea uniform
    in [1e4, 2e5] J/mol, reactant / product stoichiometry as above."""
    rng = np.random.default_rng(seed)
    A = 10.0 ** rng.uniform(8.0, 12.0, N_REACTIONS)
    Ea = rng.uniform(1e4, 2e5, N_REACTIONS)
    return {"A": A, "Ea": Ea, "nu_r": NU_REACTANTS.copy(), "nu_p": NU_PRODUCTS.copy()}


def reacting_fields(xyz, seed: int = 3005, L: float = 0.01, n_cells: int = 32, n_spheres: int = 4):
    """Seeded smooth front indicator S in [0, 1] (tanh fronts of seeded
    periodic spheres, width 4 h) and a smooth periodic velocity field of
    amplitude 1 m/s at node coordinates.  Returns (S, u, v, w)."""
    rng = np.random.default_rng(seed)
    h = L / n_cells
    centers = rng.uniform(0.0, L, (n_spheres, 3))
    radii = rng.uniform(0.15 * L, 0.3 * L, n_spheres)
    S = np.zeros(xyz.shape[:-1])
    for c, r in zip(centers, radii):
        d = xyz - c
        d = (d + 0.5 * L) % L - 0.5 * L
        dist = np.sqrt((d * d).sum(-1))
        S = np.maximum(S, 0.5 * (1.0 - np.tanh((dist - r) / (4.0 * h))))
    k = rng.integers(1, 3, (3, 3))
    ph = rng.uniform(0, 2 * math.pi, (3,))
    u = np.sin(2 * math.pi * (xyz @ k[0].astype(float)) / L + ph[0])
    v = np.sin(2 * math.pi * (xyz @ k[1].astype(float)) / L + ph[1])
    w = np.sin(2 * math.pi * (xyz @ k[2].astype(float)) / L + ph[2])
    return S, u, v, w


# Endpoints of the reacting state: a cold fuel/oxidizer/inert mixture and a
# hot product mixture.  The internal energies and densities are those of the
# default seeded species table at about 300 K and 2200 K and 1 atm; the state
# blends them along the front indicator, so each solver's own Newton solve
# yields a temperature field of roughly 300..2200 K.
Y_COLD = np.array([0.06, 0.22, 0.0, 0.0, 0.0, 0.0, 0.72])
Y_HOT = np.array([0.005, 0.04, 0.03, 0.02, 0.06, 0.125, 0.72])
E_COLD, E_HOT = 1.7934e5, -1.9697e5      # J/kg
RHO_COLD, RHO_HOT = 1.0926, 0.17571      # kg/m^3


def reacting_state(xyz, seed: int = 3005, L: float = 0.01, n_cells: int = 32):
    """Conserved reacting state q[12][...] = (rho, rho u, rho v, rho w, E,
    rho Y_1 .. rho Y_7): density, internal energy and mass fractions blended
    between the cold and hot endpoints along a seeded front, plus a seeded
    velocity field; E = rho (e + |u|^2 / 2)."""
    S, u, v, w = reacting_fields(xyz, seed, L, n_cells)
    rho = RHO_COLD * (1.0 - S) + RHO_HOT * S
    e = E_COLD * (1.0 - S) + E_HOT * S
    Y = (1.0 - S)[None] * Y_COLD.reshape((-1,) + (1,) * S.ndim) + S[None] * Y_HOT.reshape((-1,) + (1,) * S.ndim)
    E = rho * (e + 0.5 * (u * u + v * v + w * w))
    q = np.concatenate([np.stack([rho, rho * u, rho * v, rho * w, E]), rho[None] * Y], axis=0)
    return np.ascontiguousarray(q)


def shock_slab_state(xyz, rho_in: float = 120.0, rho_out: float = 1.2, x0: float = 2.5, x1: float = 7.5,
                     ripple: float = 0.3, L: float = 10.0, gamma: float = GAMMA):
    """Gas at rest with a density discontinuity: rho_in inside the slab
    x0 + r(y, z) < x < x1 + r(y, z), rho_out outside, r a rippled interface
    offset ripple sin(2 pi y / L) cos(2 pi z / L), and the pressure of the
    isentropic relation p = rho / gamma (the initial condition of the
    paper's shock / boundary-layer case, Sec. 5.3, on a periodic box)."""
    r = ripple * np.sin(2 * math.pi * xyz[..., 1] / L) * np.cos(2 * math.pi * xyz[..., 2] / L)
    x = xyz[..., 0]
    rho = np.where((x > x0 + r) & (x < x1 + r), rho_in, rho_out)
    zero = np.zeros_like(rho)
    return np.ascontiguousarray(primitive_to_conserved(rho, zero, zero, zero, rho / gamma, gamma))
