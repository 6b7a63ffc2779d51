"""Edge cases and degenerate cases of the HIP path against the oracle (run on an MI355X).

* a single periodic charge (its energy is the simple-cubic self-energy
  constant, a closed form) and a system without sites;
* vertex weights (every site fixed to one form: the correction vanishes and
  the result is the fixed-charge FMM of those charges), one-form sites,
  off-simplex weights;
* the largest site the library accepts (32 atoms, 16 forms);
* a dense cluster (leaves of several hundred atoms: many near-field passes per
  leaf), an open system confined to a slab (most leaves empty);
* coordinates outside the periodic cell and exactly on its faces.
Relative RMS ||a - b|| / ||b|| throughout; tolerances as in the main parity tests.
"""
import numpy as np
import pytest

from oracle import hi
from synth import Site, System, make_system

pytestmark = pytest.mark.gpu
KE = hi.KE_DEFAULT
XI_SC = -2.837297479480620  # lim r->0 (phi_EW(r) - 1/r) * L for the simple cubic lattice


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run(s, precision, order, depth, **kw):
    import paper_2410_01754_amd as pkg
    print(f"[gpu] {s.name} N={s.n_atoms} p={order} d={depth} prec={precision}", flush=True)
    m = pkg.from_system(s, precision=precision, order=order, depth=depth)
    out = m.eval(s.x, **kw)
    m.close()
    return out


def plain(x, q, box, periodic, precision, order, depth):
    import paper_2410_01754_amd as pkg
    m = pkg.Mahi(box, periodic, q, [], order=order, depth=depth, precision=precision)
    out = m.eval(x)
    m.close()
    return out


@pytest.mark.parametrize("pos,depth,tol,tol_f", [((1.0, 1.0, 1.0), 0, 1e-10, 1e-10),
                                                 ((1.13, 0.87, 1.21), 2, 1e-5, 1e-4),
                                                 ((0.13, 1.71, 0.52), 0, 1e-5, 1e-4),
                                                 ((0.13, 1.71, 0.52), 2, 1e-5, 1e-4)])
def test_single_periodic_charge(pos, depth, tol, tol_f):
    """E = ke q^2 xi / (2 L) for one charge in a periodic cube (neutralising
    background); F = 0 by symmetry.  At depth 0 and the cube centre the lattice
    expansion is evaluated at its own centre (exact but for rounding); elsewhere
    the result carries the order-12 truncation.  (At depth > 0 the cube centre is
    a corner of eight leaves, the worst case of the well-separation-1 bound:
    1e-3 at order 12, so the depth-2 cases use positions off the leaf grid.)
    The force, the gradient of the truncated expansions with no averaging over
    atoms, is held to ten times the energy tolerance (in units of ke q^2 / L^2)."""
    L, q = 2.0, 1.3
    s = System("single", True, L, np.array([pos], dtype=np.float32), np.array([q]), [], depth, 12, 0)
    g = run(s, 64, 12, depth)
    E = 0.5 * KE * q * q * XI_SC / L
    assert abs(g["energy"] - E) <= tol * abs(E)
    assert np.abs(g["forces"]).max() <= tol_f * KE * q * q / L ** 2


def test_no_sites_matches_oracle():
    s = make_system(300, 2.1, True, [], [], depth=2, seed=51, name="nosite")
    E, F, _, _ = hi.evaluate(s)
    g = run(s, 64, 12, 2)
    assert abs(g["energy"] - E) <= 1e-5 * abs(E)
    assert rel(g["forces"], F) <= 1e-5


def test_vertex_weights_reduce_to_fixed_charges():
    """Every site fixed to one form: covariance zero, so MAHI returns the plain FMM
    of those charges (same tree, same kernels) to rounding; dE/dlambda-tilde
    against the oracle."""
    base = make_system(300, 2.2, True, [6, 5, 7], [2, 3, 2], total_step=None, depth=2, seed=52, name="vertex")
    rng = np.random.default_rng(9)
    lam = []
    for st in base.sites:
        v = np.zeros(st.charges.shape[0])
        v[rng.integers(0, v.shape[0])] = 1.0
        lam.append(v)
    s = base.with_lam(np.concatenate(lam))
    qfix, _ = hi.scaled_charges(s.n_atoms, s.q, s.sites)
    g = run(s, 64, 12, 2)
    p = plain(s.x, qfix, s.box, True, 64, 12, 2)
    assert abs(g["energy"] - p["energy"]) <= 1e-12 * abs(p["energy"])
    assert rel(g["forces"], p["forces"]) <= 1e-12
    E, F, dv, _ = hi.evaluate(s)
    assert rel(g["dvdl"], dv) <= 1e-5


def test_one_form_sites_and_off_simplex_weights():
    """One-form sites (no interpolation) beside two- and three-form sites whose
    weights are off the simplex (the general formulation stays exact there)."""
    base = make_system(250, 2.0, True, [4, 6, 5], [1, 2, 3], total_step=None, depth=2, seed=53, name="offsimplex")
    s = base.with_lam(np.array([1.0, 0.7, 0.6, 0.5, -0.2, 0.9]))
    E, F, dv, dq = hi.evaluate(s)
    g = run(s, 64, 12, 2, dedq=True)
    assert abs(g["energy"] - E) <= 1e-5 * abs(E)
    assert rel(g["forces"], F) <= 1e-5 and rel(g["dvdl"], dv) <= 1e-5
    assert rel(g["dedq"], np.concatenate([d.reshape(-1) for d in dq])) <= 1e-5


@pytest.mark.parametrize("periodic,prec,depth,tol", [(False, 64, 0, 1e-12), (False, 64, 2, 1e-5),
                                                     (False, 32, 2, 2e-4), (True, 64, 2, 1e-5),
                                                     (True, 32, 2, 2e-4)])
def test_largest_site(periodic, prec, depth, tol):
    """A 32-atom, 16-form site (the largest accepted; its work arrays exceed local
    memory and live in the global workspace) and a one-atom, one-form site."""
    rng = np.random.default_rng(54)
    n_env = 200
    x = rng.random((n_env + 33, 3)) * 2.0
    q = np.concatenate([rng.uniform(-0.8, 0.8, n_env), np.zeros(33)])
    big = Site(np.arange(n_env, n_env + 32), rng.uniform(-0.9, 0.9, (16, 32)), rng.dirichlet(np.ones(16)))
    one = Site(np.array([n_env + 32]), np.array([[0.4]]), np.array([1.0]))
    s = System("bigsite", periodic, 2.0, x.astype(np.float32), q, [big, one], depth, 12, 54)
    E, F, dv, _ = hi.evaluate(s)
    g = run(s, prec, 12 if prec == 64 else 8, depth)
    print("bigsite", periodic, prec, depth, abs(g["energy"] - E) / abs(E), rel(g["forces"], F), rel(g["dvdl"], dv))
    assert abs(g["energy"] - E) <= tol * abs(E)
    assert rel(g["forces"], F) <= tol and rel(g["dvdl"], dv) <= tol


@pytest.mark.parametrize("prec,order,tol", [(64, 12, 1e-5), (32, 8, 2e-4)])
def test_dense_cluster_many_passes(prec, order, tol):
    """400 atoms packed into a 0.35 nm ball inside a water box: the leaf holding
    them needs several passes of 64 targets, against sources of the same size."""
    rng = np.random.default_rng(55)
    base = make_system(300, 2.2, True, [6, 5], [2, 2], total_step=None, depth=2, seed=55, name="cluster")
    n_c = 400
    d = rng.normal(size=(n_c, 3))
    d *= (0.35 * rng.random(n_c) ** (1 / 3) / np.linalg.norm(d, axis=1))[:, None]
    xc = (np.array([0.9, 1.1, 1.0]) + d).astype(np.float32)
    qc = rng.uniform(-0.5, 0.5, n_c)
    s = System("cluster", True, base.box, np.concatenate([base.x, xc]), np.concatenate([base.q, qc]), base.sites,
               2, order, 55)
    E, F, dv, _ = hi.hi_periodic(s.x, s.q, s.sites, s.box)
    g = run(s, prec, order, 2)
    print("cluster", prec, abs(g["energy"] - E) / abs(E), rel(g["forces"], F), rel(g["dvdl"], dv))
    assert abs(g["energy"] - E) <= tol * abs(E)
    assert rel(g["forces"], F) <= tol and rel(g["dvdl"], dv) <= tol


def test_open_slab_mostly_empty_leaves():
    """Open boundaries with every atom in a thin slab: at depth 3 most leaves are empty."""
    rng = np.random.default_rng(56)
    x = np.column_stack([rng.random(600) * 3.0, rng.random(600) * 3.0, 1.0 + 0.05 * rng.random(600)])
    q = rng.uniform(-0.8, 0.8, 600)
    q[-4:] = 0.0
    st = Site(np.arange(596, 600), rng.uniform(-0.8, 0.8, (2, 4)), np.array([0.3, 0.7]))
    s = System("slab", False, 3.0, x.astype(np.float32), q, [st], 3, 12, 56)
    E, F, dv, _ = hi.evaluate(s)
    g = run(s, 64, 12, 3)
    assert abs(g["energy"] - E) <= 1e-5 * abs(E)
    assert rel(g["forces"], F) <= 1e-5 and rel(g["dvdl"], dv) <= 1e-5


@pytest.mark.parametrize("prec", [64, 32])
def test_coordinates_outside_the_cell(prec):
    """Shifting atoms by whole cells, or onto the cell faces, changes nothing
    beyond the rounding of the wrap."""
    s = make_system(300, 2.4, True, [6, 5], [2, 2], total_step=None, depth=2, seed=57, name="wrap")
    dt = np.float32 if prec == 32 else np.float64
    x0 = s.x.astype(dt)
    rng = np.random.default_rng(7)
    shift = rng.integers(-3, 4, size=x0.shape).astype(dt) * dt(s.box)
    x1 = x0 + shift
    a = run(s, prec, 8, 2)
    s1 = System(s.name, True, s.box, x1, s.q, s.sites, 2, 8, s.seed)
    b = run(s1, prec, 8, 2)
    tol = 1e-12 if prec == 64 else 2e-5
    assert abs(a["energy"] - b["energy"]) <= tol * abs(a["energy"])
    assert rel(b["forces"], a["forces"]) <= tol and rel(b["dvdl"], a["dvdl"]) <= tol
    # an atom exactly on the lower face and one exactly on the upper face (wraps to 0)
    x2 = x0.copy()
    x2[0] = (0.0, 0.0, 0.0)
    x2[1] = (s.box, 0.5, 0.5)
    s2 = System(s.name, True, s.box, x2, s.q, s.sites, 2, 8, s.seed)
    x3 = x2.copy()
    x3[1] = (0.0, 0.5, 0.5)
    s3 = System(s.name, True, s.box, x3, s.q, s.sites, 2, 8, s.seed)
    c, d = run(s2, prec, 8, 2), run(s3, prec, 8, 2)
    if prec == 64:
        # L itself wraps to exactly 0
        assert c["energy"] == d["energy"] and np.array_equal(c["forces"], d["forces"])
    else:
        # float32(L) lies one rounding step above L and wraps to ~1e-7 nm
        assert abs(c["energy"] - d["energy"]) <= tol * abs(d["energy"]) and rel(c["forces"], d["forces"]) <= tol
