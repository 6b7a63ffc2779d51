"""Seeded synthetic water-like systems with titratable sites.

The paper measures on random particle systems (Accuracy and Performance
Assessment, "Random Systems"): environment charges plus a few titratable
sites whose forms carry different partial charges.  The generators here build
stand-ins with water-like shapes and densities:

* rigid 3-site waters: O at a uniform random point, two H at 0.09572 nm with an
  H-O-H angle of 104.52 degrees, oriented by a uniform random rotation (Shoemake
  quaternion); charges O -0.834 e, H +0.417 e;
* sites of n atoms, either clustered (uniform in a 0.3 nm ball around a uniform
  centre, at least 0.1 nm apart, the paper's "typical case") or spread uniformly
  through the box (the paper's "worst case");
* per-form charges drawn uniformly from [lo, hi]; optionally the form totals are
  forced to differ by exactly 1 e (form rho+1 carries one elementary charge less
  than form rho);
* weights lambda-tilde per site: (1 - lam, lam) with lam ~ U[0,1] for two-form
  sites, or uniform on the simplex (Dirichlet(1,...,1)).

All coordinates are generated in float64 and rounded once to float32; both the
GPU path and the oracle consume these identical float32 values.  Periodic
systems are wrapped into [0, L) before rounding, and a coordinate that rounds to
L is mapped to 0.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

OH_NM = 0.09572
HOH_DEG = 104.52
Q_O = -0.834
Q_H = 0.417
WATER_DENSITY = 33.4  # waters per nm^3


@dataclass
class Site:
    atoms: np.ndarray          # int64 [n], indices into the atom arrays
    charges: np.ndarray        # float64 [n_forms, n], charge of every atom in every form
    lam: np.ndarray            # float64 [n_forms], lambda-tilde weights


@dataclass
class System:
    name: str
    periodic: bool
    box: float                 # cube edge (nm); open systems: edge of the cube the waters were drawn in
    x: np.ndarray              # float32 [N, 3]
    q: np.ndarray              # float64 [N]; environment charges, 0 at site atoms
    sites: List[Site] = field(default_factory=list)
    depth: int = 0
    order: int = 8
    seed: int = 0

    @property
    def n_atoms(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_forms(self) -> int:
        return int(sum(s.charges.shape[0] for s in self.sites))

    def lam_flat(self) -> np.ndarray:
        if not self.sites:
            return np.zeros(0)
        return np.concatenate([s.lam for s in self.sites])

    def with_lam(self, lam_flat) -> "System":
        """Copy with new lambda-tilde weights (flat, site-major)."""
        lam_flat = np.asarray(lam_flat, dtype=np.float64)
        sites, o = [], 0
        for s in self.sites:
            f = s.charges.shape[0]
            sites.append(Site(s.atoms.copy(), s.charges.copy(), lam_flat[o:o + f].copy()))
            o += f
        return System(self.name, self.periodic, self.box, self.x.copy(), self.q.copy(), sites,
                      self.depth, self.order, self.seed)


def random_rotations(n: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation matrices via Shoemake's quaternion method."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    qx = a * np.sin(2 * np.pi * u2)
    qy = a * np.cos(2 * np.pi * u2)
    qz = b * np.sin(2 * np.pi * u3)
    qw = b * np.cos(2 * np.pi * u3)
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (qy * qy + qz * qz)
    R[:, 0, 1] = 2 * (qx * qy - qz * qw)
    R[:, 0, 2] = 2 * (qx * qz + qy * qw)
    R[:, 1, 0] = 2 * (qx * qy + qz * qw)
    R[:, 1, 1] = 1 - 2 * (qx * qx + qz * qz)
    R[:, 1, 2] = 2 * (qy * qz - qx * qw)
    R[:, 2, 0] = 2 * (qx * qz - qy * qw)
    R[:, 2, 1] = 2 * (qy * qz + qx * qw)
    R[:, 2, 2] = 1 - 2 * (qx * qx + qy * qy)
    return R


def water_geometry() -> np.ndarray:
    """Body-frame offsets of the two H atoms from O (nm), shape [2, 3]."""
    half = np.deg2rad(HOH_DEG) / 2.0
    return np.array([[OH_NM * np.sin(half), 0.0, OH_NM * np.cos(half)],
                     [-OH_NM * np.sin(half), 0.0, OH_NM * np.cos(half)]])


def waters(n: int, edge: float, rng: np.random.Generator):
    """n rigid waters with O uniform in [0, edge)^3; returns (x [3n,3] f64, q [3n])."""
    o = rng.random((n, 3)) * edge
    R = random_rotations(n, rng)
    hb = water_geometry()
    h1 = o + R @ hb[0]
    h2 = o + R @ hb[1]
    x = np.empty((3 * n, 3))
    x[0::3], x[1::3], x[2::3] = o, h1, h2
    q = np.empty(3 * n)
    q[0::3], q[1::3], q[2::3] = Q_O, Q_H, Q_H
    return x, q


def clustered_positions(n: int, edge: float, rng: np.random.Generator,
                        radius: float = 0.3, min_dist: float = 0.1) -> np.ndarray:
    centre = rng.random(3) * edge
    pts: list = []
    for _attempt in range(1000000):
        if len(pts) == n:
            break
        d = rng.uniform(-radius, radius, 3)
        if d @ d > radius * radius:
            continue
        p = centre + d
        if all(np.linalg.norm(p - o) >= min_dist for o in pts):
            pts.append(p)
    if len(pts) < n:
        raise ValueError("clustered site: cannot place atoms")
    return np.array(pts)


def form_charges(n_forms: int, n: int, lo: float, hi: float, rng: np.random.Generator,
                 total_step: Optional[float]) -> np.ndarray:
    """Charges [n_forms, n] uniform in [lo, hi].

    With total_step set, form rho carries sum(q^0) - rho * total_step in total;
    each later form is drawn, shifted by a constant to meet its total, and
    redrawn until every charge lies inside [lo, hi].
    """
    out = np.empty((n_forms, n))
    out[0] = rng.uniform(lo, hi, n)
    for r in range(1, n_forms):
        for _attempt in range(100000):
            c = rng.uniform(lo, hi, n)
            if total_step is not None:
                c = c + ((out[0].sum() - r * total_step) - c.sum()) / n
            if np.all(c >= lo) and np.all(c <= hi):
                out[r] = c
                break
        else:
            raise ValueError("form charges: total rule cannot be met inside [lo, hi]")
    return out


def lam_two_form(rng: np.random.Generator) -> np.ndarray:
    lam = rng.random()
    return np.array([1.0 - lam, lam])


def lam_simplex(n_forms: int, rng: np.random.Generator) -> np.ndarray:
    return rng.dirichlet(np.ones(n_forms))


def _finish(name, periodic, edge, xw, qw, site_specs, depth, order, seed) -> System:
    """Append site atoms after the waters, wrap (periodic) and round to float32."""
    xs, sites, n0 = [xw], [], xw.shape[0]
    for pos, charges, lam in site_specs:
        idx = np.arange(n0, n0 + pos.shape[0])
        n0 += pos.shape[0]
        xs.append(pos)
        sites.append(Site(idx, charges, lam))
    x = np.concatenate(xs)
    if periodic:
        x = x - edge * np.floor(x / edge)
    x32 = x.astype(np.float32)
    if periodic:
        x32[x32 >= np.float32(edge)] = np.float32(0.0)
        x32[x32 < 0] = np.float32(0.0)
    q = np.concatenate([qw, np.zeros(x.shape[0] - qw.shape[0])])
    return System(name, periodic, float(edge), x32, q, sites, depth, order, seed)


def make_system(n_waters: int, edge: float, periodic: bool, site_sizes, site_forms,
                qrange=(-0.8, 0.8), total_step: Optional[float] = 1.0, clustered=True,
                simplex=False, depth=2, order=8, seed=0, name="custom") -> System:
    """General recipe used by the named configurations and by the tests."""
    rng = np.random.default_rng(seed)
    xw, qw = waters(n_waters, edge, rng)
    specs = []
    for n, f in zip(site_sizes, site_forms):
        pos = clustered_positions(n, edge, rng) if clustered else rng.random((n, 3)) * edge
        ch = form_charges(f, n, qrange[0], qrange[1], rng, total_step)
        lam = lam_simplex(f, rng) if (simplex or f != 2) else lam_two_form(rng)
        specs.append((pos, ch, lam))
    return _finish(name, periodic, edge, xw, qw, specs, depth, order, seed)


CONFIG_NAMES = {
    0: "open 2.2 nm, 333 waters + 4 two-form sites of 5 atoms (spread), d=2, p=8",
    1: "periodic 10.0 nm, 33,400 waters + 64 sites (48 two-form, 16 three-form, 6-10 atoms), d=4, p=8",
    2: "periodic 21.5 nm, 333,400 waters + 512 two-form sites of 8 atoms, d=5, p=8",
}


def make_config(k: int, seed: Optional[int] = None) -> System:
    """The named workloads; seed defaults to 1754 + k."""
    seed = 1754 + k if seed is None else seed
    rng = np.random.default_rng(seed)
    if k == 0:
        edge = 2.2
        xw, qw = waters(333, edge, rng)
        specs = []
        for _ in range(4):
            pos = rng.random((5, 3)) * edge
            ch = form_charges(2, 5, -0.8, 0.8, rng, 1.0)
            specs.append((pos, ch, lam_two_form(rng)))
        return _finish("config0", False, edge, xw, qw, specs, 2, 8, seed)
    if k == 1:
        edge = 10.0
        xw, qw = waters(33400, edge, rng)
        specs = []
        for s in range(64):
            nf = 2 if s < 48 else 3
            n = int(rng.integers(6, 11))
            pos = clustered_positions(n, edge, rng)
            ch = form_charges(nf, n, -0.9, 0.9, rng, None)
            specs.append((pos, ch, lam_simplex(nf, rng)))
        return _finish("config1", True, edge, xw, qw, specs, 4, 8, seed)
    if k == 2:
        edge = 21.5
        xw, qw = waters(333400, edge, rng)
        specs = []
        for _ in range(512):
            pos = clustered_positions(8, edge, rng)
            ch = form_charges(2, 8, -0.8, 0.8, rng, 1.0)
            specs.append((pos, ch, lam_two_form(rng)))
        return _finish("config2", True, edge, xw, qw, specs, 5, 8, seed)
    raise ValueError(f"unknown configuration {k}")


def make_batch(n_systems: int = 96, n_min: int = 3000, n_max: int = 60000, seed: int = 1758,
               depth: int = 3, order: int = 8) -> list:
    """Many small periodic water boxes (the paper's small-system regime): total
    atom counts log-uniform in [n_min, n_max], edge (N_w / 33.4)^(1/3) nm, 4..64
    clustered two-form sites of 6..10 atoms, lambda ~ U[0, 1].  depth and order
    are placeholders; callers choose their own per system.  The two forms of a
    site are drawn independently (no total rule)."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n_systems):
        n_tot = float(np.exp(rng.uniform(np.log(n_min), np.log(n_max))))
        n_sites = int(rng.integers(4, 65))
        sizes = rng.integers(6, 11, size=n_sites)
        n_w = max(1, int(round((n_tot - sizes.sum()) / 3)))
        edge = (n_w / 33.4) ** (1.0 / 3.0)
        xw, qw = waters(n_w, edge, rng)
        specs = []
        for n in sizes:
            pos = clustered_positions(int(n), edge, rng)
            ch = form_charges(2, int(n), -0.8, 0.8, rng, None)
            specs.append((pos, ch, lam_two_form(rng)))
        out.append(_finish(f"batch{b}", True, edge, xw, qw, specs, depth, order, seed * 1000 + b))
    return out
