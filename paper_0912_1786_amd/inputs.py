"""Seeded synthetic initial conditions for the Tree+SPH force engine.

This module draws particle sets only: positions, velocities, masses and
internal energies.  It holds none of the method's arithmetic (no kernel, no
tree, no force), so both the HIP path and the FP64 oracle consume the same
bytes from it.

Random numbers come from a counter-based generator built on the SplitMix64
finaliser (Steele, Lea & Flood 2014, "Fast splittable pseudorandom number
generators"): the value for (seed, stream, index) is the finaliser applied to
a per-(seed, stream) key plus (index + 1) times the golden-ratio increment.
Uniform doubles take the top 53 bits.

Workloads (code units G = M = R = 1):

* ``evrard``     -- gas sphere with rho ~ 1/r (Evrard 1988 collapse, Sect. 5
  "Self-gravitating collapse"): r = sqrt(X) so that M(<r) = r^2, isotropic
  directions, equal masses 1/N, zero velocity, u = u0.
* ``plummer``    -- Plummer sphere rho ~ (1 + r^2/a^2)^(-5/2) (Sect. 5
  "Collision of two gas spheres"; the printed (1+r)^(-5/2) is read as the
  usual Plummer law), radii by the inverse mass profile, truncated at
  ``rmax_over_a`` scale radii.
* ``two_species_field`` -- 64 Plummer halos of dark matter and gas in a unit
  cube (DM:gas particle mass 5:1), halo masses from dN/dM ~ M^-1.9, scale radii
  log-uniform in [0.01, 0.1], isotropic Gaussian velocities with the Plummer
  dispersion, gas u log-uniform in [1e-3, 1e-1].
* ``lattice``    -- simple-cubic and two-lattice (BCC) arrangements used by the
  density tests (Sect. 3, mixed-mass density-determination test).

Every generator returns a dict of float64 numpy arrays in *caller order*: gas
particles first (indices [0, n_gas)), then dark matter.
"""
from __future__ import annotations

import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser, applied elementwise to uint64 arrays."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def rand_u64(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """n raw 64-bit values for (seed, stream), counter = offset .. offset+n-1."""
    with np.errstate(over="ignore"):
        key = _mix64(np.array([np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * _GOLDEN
                               + np.uint64(stream & 0xFFFFFFFF)], dtype=np.uint64))[0]
        ctr = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        return _mix64(key + ctr * _GOLDEN)


def uniform(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits."""
    return (rand_u64(seed, stream, n, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_open(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in (0, 1)."""
    return ((rand_u64(seed, stream, n, offset) >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)


def normal(seed: int, stream: int, n: int) -> np.ndarray:
    """Standard normal deviates (Box-Muller on two uniform streams)."""
    u1 = uniform_open(seed, stream, n)
    u2 = uniform(seed, stream + 0x10000, n)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def _isotropic(seed: int, stream: int, n: int):
    cth = 2.0 * uniform(seed, stream, n) - 1.0
    phi = 2.0 * math.pi * uniform(seed, stream + 1, n)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    return sth * np.cos(phi), sth * np.sin(phi), cth


def _pack(x, y, z, vx, vy, vz, m, u, n_gas, **extra):
    d = dict(x=np.ascontiguousarray(x, np.float64), y=np.ascontiguousarray(y, np.float64),
             z=np.ascontiguousarray(z, np.float64), vx=np.ascontiguousarray(vx, np.float64),
             vy=np.ascontiguousarray(vy, np.float64), vz=np.ascontiguousarray(vz, np.float64),
             m=np.ascontiguousarray(m, np.float64), u=np.ascontiguousarray(u, np.float64),
             n=int(len(x)), n_gas=int(n_gas))
    d.update(extra)
    return d


def evrard(n: int, seed: int = 1, u0: float = 0.05, v_sigma: float = 0.0) -> dict:
    """Evrard sphere: M = R = 1, rho ~ 1/r, all gas, u = u0.

    ``v_sigma`` > 0 adds isotropic Gaussian velocities (each component
    N(0, v_sigma^2)) so that the artificial viscosity is exercised.
    """
    r = np.sqrt(uniform(seed, 0, n))
    ex, ey, ez = _isotropic(seed, 1, n)
    x, y, z = r * ex, r * ey, r * ez
    if v_sigma > 0.0:
        vx = v_sigma * normal(seed, 10, n)
        vy = v_sigma * normal(seed, 11, n)
        vz = v_sigma * normal(seed, 12, n)
    else:
        vx = vy = vz = np.zeros(n)
    m = np.full(n, 1.0 / n)
    u = np.full(n, float(u0))
    return _pack(x, y, z, vx, vy, vz, m, u, n_gas=n, workload="evrard", seed=seed)


def plummer_radii(seed: int, stream: int, n: int, a: float, rmax_over_a: float = 5.0) -> np.ndarray:
    """Radii from the Plummer cumulative mass M(<r)/M = r^3/(r^2+a^2)^(3/2),
    inverted as r = a (X^(-2/3) - 1)^(-1/2), with X restricted to the mass
    inside rmax so that no particle lies beyond it."""
    c = rmax_over_a
    xmax = c ** 3 / (c * c + 1.0) ** 1.5
    X = xmax * uniform_open(seed, stream, n)
    return a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)


def plummer(n: int, seed: int = 1, a: float = 1.0, mass: float = 1.0, n_gas: int | None = None,
            u0: float = 0.05, rmax_over_a: float = 5.0, velocities: bool = False) -> dict:
    """Single Plummer sphere of total mass ``mass``; the first ``n_gas`` particles are gas."""
    if n_gas is None:
        n_gas = n
    r = plummer_radii(seed, 0, n, a, rmax_over_a)
    ex, ey, ez = _isotropic(seed, 1, n)
    if velocities:
        sig = np.sqrt(mass / (6.0 * np.sqrt(r * r + a * a)))
        vx, vy, vz = (sig * normal(seed, 10 + k, n) for k in range(3))
    else:
        vx = vy = vz = np.zeros(n)
    m = np.full(n, mass / n)
    u = np.where(np.arange(n) < n_gas, u0, 0.0)
    return _pack(r * ex, r * ey, r * ez, vx, vy, vz, m, u, n_gas=n_gas, workload="plummer", seed=seed)


def _largest_remainder(weights: np.ndarray, total: int) -> np.ndarray:
    w = np.asarray(weights, np.float64)
    quota = w / w.sum() * total
    base = np.floor(quota).astype(np.int64)
    rem = total - int(base.sum())
    order = np.lexsort((np.arange(len(w)), -(quota - base)))
    base[order[:rem]] += 1
    return base


def halo_catalogue(n_halo: int, seed: int):
    """Centres U[0,1]^3, scale radii 10^U(-2,-1), masses from dN/dM ~ M^-1.9
    on [1, 100] (inverse CDF), normalised to a total of 1."""
    centres = np.stack([uniform(seed, 100 + k, n_halo) for k in range(3)], axis=1)
    a = 10.0 ** (-2.0 + uniform(seed, 103, n_halo))
    s = 1.0 - 1.9  # exponent of the cumulative
    lo, hi = 1.0, 100.0
    X = uniform(seed, 104, n_halo)
    M = (lo ** s + X * (hi ** s - lo ** s)) ** (1.0 / s)
    return centres, a, M / M.sum()


def two_species_field(n_dm: int = 1 << 20, n_gas: int = 1 << 20, n_halo: int = 64, seed: int = 1,
                      mass_ratio: float = 5.0) -> dict:
    """Clustered field of gas + dark matter in ``n_halo`` Plummer halos.

    The same particle count per halo is used for both species (proportional to
    the halo mass, largest-remainder rounding).  Total mass is 1; a DM particle
    weighs ``mass_ratio`` gas particles.  Gas comes first in the returned arrays.
    """
    if n_dm != n_gas:
        raise ValueError("two_species_field draws equal gas and DM counts per halo")
    centres, a, M = halo_catalogue(n_halo, seed)
    counts = _largest_remainder(M, n_gas)
    m_gas = 1.0 / (n_gas * (1.0 + mass_ratio))
    m_dm = mass_ratio * m_gas
    halo_of = np.repeat(np.arange(n_halo), counts)
    out = {}
    for sp, (stream0, n_sp) in enumerate(((200, n_gas), (300, n_dm))):
        r = np.empty(n_sp)
        for k in range(n_halo):
            sel = halo_of == k
            r[sel] = plummer_radii(seed * 1000003 + k, stream0, int(counts[k]), a[k])
        ex, ey, ez = _isotropic(seed, stream0 + 1, n_sp)
        c = centres[halo_of]
        x = c[:, 0] + r * ex
        y = c[:, 1] + r * ey
        z = c[:, 2] + r * ez
        mh = counts[halo_of] * (m_gas + m_dm)
        sig = np.sqrt(mh / (6.0 * np.sqrt(r * r + a[halo_of] ** 2)))
        v = [sig * normal(seed, stream0 + 10 + k, n_sp) for k in range(3)]
        out[sp] = (x, y, z, v[0], v[1], v[2])
    cat = lambda i: np.concatenate([out[0][i], out[1][i]])
    m = np.concatenate([np.full(n_gas, m_gas), np.full(n_dm, m_dm)])
    u = np.concatenate([10.0 ** (-3.0 + 2.0 * uniform(seed, 400, n_gas)), np.zeros(n_dm)])
    return _pack(cat(0), cat(1), cat(2), cat(3), cat(4), cat(5), m, u, n_gas=n_gas,
                 workload="two_species_field", seed=seed)


def ensemble_sizes(n_sim: int = 256, seed: int = 1, lo_log2: float = 10.0, hi_log2: float = 15.0):
    """Member sizes N_k = round(2^U(lo, hi)) and u0_k = U(0.02, 0.1)."""
    nk = np.rint(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * uniform(seed, 500, n_sim))).astype(np.int64)
    u0 = 0.02 + 0.08 * uniform(seed, 501, n_sim)
    return nk, u0


def cubic_lattice(n_side: int, spacing: float = 1.0, mass: float = 1.0, jitter: float = 0.0,
                  seed: int = 1) -> dict:
    """n_side^3 simple-cubic lattice; all gas; optional uniform jitter of the given amplitude."""
    g = (np.arange(n_side) + 0.5) * spacing
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy()
    n = x.size
    if jitter > 0:
        x += jitter * (uniform(seed, 600, n) - 0.5)
        y += jitter * (uniform(seed, 601, n) - 0.5)
        z += jitter * (uniform(seed, 602, n) - 0.5)
    zero = np.zeros(n)
    return _pack(x, y, z, zero, zero, zero, np.full(n, mass), np.full(n, 1.0), n_gas=n,
                 workload="cubic_lattice", seed=seed)


def random_cloud(n: int, seed: int = 1, masses=(1.0, 5.0), n_gas: int | None = None,
                 v_sigma: float = 0.1, u_range=(0.5, 1.5)) -> dict:
    """Uniform cloud in the unit cube with two particle masses (normalised so
    that the total mass is 1) and small random velocities; used by the
    finite-difference tests."""
    if n_gas is None:
        n_gas = n
    x, y, z = (uniform(seed, 700 + k, n) for k in range(3))
    pick = uniform(seed, 703, n) < 0.5
    m = np.where(pick, masses[0], masses[1]).astype(np.float64)
    m /= m.sum()
    vx, vy, vz = (v_sigma * normal(seed, 710 + k, n) for k in range(3))
    u = np.where(np.arange(n) < n_gas, u_range[0] + (u_range[1] - u_range[0]) * uniform(seed, 704, n), 0.0)
    return _pack(x, y, z, vx, vy, vz, m, u, n_gas=n_gas, workload="random_cloud", seed=seed)


def mixed_mass_lattice(spacing: float = 0.01, lx: float = 1.0, ly: float = 0.1, lz: float = 0.1,
                       u: float = 1.0) -> dict:
    """The mixed-mass density test (Sect. 3): two simple-cubic lattices of
    the same spacing in the slab 0 < x < lx, 0 < y < ly, 0 < z < lz, the
    second shifted by half a spacing along every axis (5e-3 for the 0.01
    spacing, as printed).  Masses per lattice and side: 0.9e-6 and 0.1e-6
    for x < 0.5, 2.25e-7 and 0.25e-7 for x >= 0.5, so that the densities are
    1 and 0.25 with a spacing of 0.01 (a reading: the spacing is not
    printed).  All gas, at rest; the heavy lattice first."""
    def grid(off):
        gx = np.arange(int(round(lx / spacing))) * spacing + off
        gy = np.arange(int(round(ly / spacing))) * spacing + off
        gz = np.arange(int(round(lz / spacing))) * spacing + off
        X, Y, Z = np.meshgrid(gx, gy, gz, indexing="ij")
        return X.ravel(), Y.ravel(), Z.ravel()
    x1, y1, z1 = grid(0.25 * spacing)
    x2, y2, z2 = grid(0.75 * spacing)
    x, y, z = np.concatenate([x1, x2]), np.concatenate([y1, y2]), np.concatenate([z1, z2])
    heavy = np.arange(x.size) < x1.size
    left = x < 0.5 * lx
    m = np.where(heavy, np.where(left, 0.9e-6, 2.25e-7), np.where(left, 0.1e-6, 0.25e-7))
    n = x.size
    zero = np.zeros(n)
    return _pack(x.copy(), y.copy(), z.copy(), zero, zero, zero, m, np.full(n, u), n_gas=n,
                 workload="mixed_mass_lattice", seed=0)
