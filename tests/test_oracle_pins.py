"""Pins of the CPU oracle against facts fixed by the paper or by mathematics.

None of these compares the oracle with itself: each pin is a brute-force
definition, a closed form, a textbook constant, an invariant or a finite
difference.  Some tests plant a mistake in the oracle (on the CPU) and check
that a pin catches it.
"""
import os

import numpy as np
import pytest

from oracle import brute, ewald, hi, kernels, lmap
from synth import Site, System, make_config, make_system

HERE = os.path.dirname(os.path.abspath(__file__))
KE = hi.KE_DEFAULT


def small(periodic, seed=5, sizes=(4, 3, 5), forms=(2, 4, 3), n_w=25, edge=1.3, clustered=True):
    return make_system(n_w, edge, periodic, list(sizes), list(forms), total_step=None, clustered=clustered,
                       depth=0, seed=seed)


def dense(s):
    return kernels.dense(s.x, s.periodic, s.box)


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ---------------------------------------------------------------- P1: brute force

@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("clustered", [False, True])
def test_general_formulation_equals_enumeration(periodic, clustered):
    """Eq iter_ham_lambda equals the weighted sum of all sub-Hamiltonians (eq rek_ham_lambda)."""
    s = small(periodic, clustered=clustered)
    Phi, G = dense(s)
    E, F, dvdl, dedq = hi.hi_dense(s.q, s.sites, Phi, G)
    Eb, Fb, dqb = brute.enumerate_hi(s.q, s.sites, Phi, G)
    assert abs(E - Eb) <= 1e-12 * abs(Eb)
    assert rel(F, Fb) <= 1e-12
    for a, b in zip(dedq, dqb):
        assert rel(a, b) <= 1e-12


def test_enumeration_catches_dropped_form_form_term(monkeypatch):
    """Planted mistake: replacing the form-form weights by the QI form must break P1."""
    s = small(False)
    Phi, G = dense(s)
    Eb = brute.enumerate_hi(s.q, s.sites, Phi, G)[0]
    qt, _ = hi.scaled_charges(s.n_atoms, s.q, s.sites)
    E_qi = 0.5 * KE * qt @ Phi @ qt
    assert abs(E_qi - Eb) > 1e-6 * abs(Eb)


# ---------------------------------------------------------------- P2: dV/dlt by deletion

@pytest.mark.parametrize("periodic", [False, True])
def test_dvdl_equals_vertex_minus_deleted(periodic):
    s = small(periodic)
    Phi, G = dense(s)
    _, _, dvdl, _ = hi.hi_dense(s.q, s.sites, Phi, G)
    ref = brute.dvdl_by_deletion(s.q, s.sites, Phi)
    assert np.max(np.abs(dvdl - ref)) <= 1e-10 * np.max(np.abs(ref))


# ---------------------------------------------------------------- P3: QI vs HI closed form

@pytest.mark.parametrize("periodic", [False, True])
def test_single_two_form_site_closed_form(periodic):
    """One two-form site: H_QI - H_HI = (k/2)(lam^2 - lam) (eq Udiff) and
    dH_QI/dlam - dH_HI/dlam = (lam - 1/2) k (eq DeltaFQIHI)."""
    base = make_system(20, 1.4, periodic, [5], [2], total_step=1.0, depth=0, seed=11)
    Phi, G = dense(base)
    st = base.sites[0]
    d = st.charges[0] - st.charges[1]
    k = d @ Phi[np.ix_(st.atoms, st.atoms)] @ d
    for lam in (0.0, 0.345, 0.721, 1.0):
        s = base.with_lam([1 - lam, lam])
        E, _, dvdl, _ = hi.hi_dense(s.q, s.sites, Phi, G)
        E_qi, dv_qi = hi.qi_dense(s.q, s.sites, Phi)
        assert abs((E_qi - E) - KE * 0.5 * k * (lam * lam - lam)) <= 1e-10 * abs(E)
        dH = dvdl[1] - dvdl[0]
        dQI = dv_qi[1] - dv_qi[0]
        assert abs((dQI - dH) - KE * (lam - 0.5) * k) <= 1e-9 * max(abs(dH), 1.0)


def test_qi_dropped_cross_term_is_caught(monkeypatch):
    """Planted mistake: a QI energy without the site-environment cross term breaks the closed form."""
    base = make_system(20, 1.4, False, [5], [2], total_step=1.0, depth=0, seed=11)
    Phi, G = dense(base)
    st = base.sites[0]
    d = st.charges[0] - st.charges[1]
    k = d @ Phi[np.ix_(st.atoms, st.atoms)] @ d
    s = base.with_lam([0.655, 0.345])
    E, _, _, _ = hi.hi_dense(s.q, s.sites, Phi, G)
    qt, site_of = hi.scaled_charges(s.n_atoms, s.q, s.sites)
    cut = np.where((site_of[:, None] >= 0) != (site_of[None, :] >= 0), 0.0, Phi)
    monkeypatch.setattr(hi, "qi_dense", lambda q, sites, P, ke=KE: (ke * 0.5 * qt @ cut @ qt, None))
    E_qi, _ = hi.qi_dense(s.q, s.sites, Phi)
    assert abs((E_qi - E) - KE * 0.5 * k * (0.345 ** 2 - 0.345)) > 1e-6 * abs(E)


def test_qi_outputs_of_hi_periodic_match_dense():
    s = small(True, seed=10)
    Phi, _ = dense(s)
    Ed, dvd = hi.qi_dense(s.q, s.sites, Phi)
    out = hi.hi_periodic(s.x, s.q, s.sites, s.box, qi=True)
    assert abs(out[4] - Ed) <= 1e-11 * abs(Ed) and rel(out[5], dvd) <= 1e-11
    part = hi.hi_periodic(s.x, s.q, s.sites, s.box, targets=[0, 1], qi=True)
    assert part[4] is None and rel(part[5], dvd) <= 1e-11


def test_qi_periodic_derivative_by_central_difference():
    """dE_QI/dlt from qi_periodic equals the central difference of its E_QI (E_QI is
    quadratic in the weights, so the difference is exact up to rounding), and the
    Ewald-field path agrees with the dense pair-kernel path."""
    s = small(True, seed=9)
    E0, dv = hi.qi_periodic(s.x, s.q, s.sites, s.box)
    Phi, _ = dense(s)
    Ed, dvd = hi.qi_dense(s.q, s.sites, Phi)
    assert abs(E0 - Ed) <= 1e-11 * abs(Ed) and rel(dv, dvd) <= 1e-11
    lam = s.lam_flat()
    h = 1e-3
    k = 0
    for si, st in enumerate(s.sites):
        for r in range(st.charges.shape[0]):
            lp, lm = lam.copy(), lam.copy()
            lp[k] += h
            lm[k] -= h
            Ep, _ = hi.qi_periodic(s.x, s.q, s.with_lam(lp).sites, s.box)
            Em, _ = hi.qi_periodic(s.x, s.q, s.with_lam(lm).sites, s.box)
            assert abs((Ep - Em) / (2 * h) - dv[k]) <= 1e-7 * max(abs(dv[k]), 1.0)
            k += 1


# ---------------------------------------------------------------- P4: vertices

@pytest.mark.parametrize("periodic", [False, True])
def test_vertex_weights_give_fixed_charge_energy(periodic):
    s0 = small(periodic)
    Phi, G = dense(s0)
    rng = np.random.default_rng(0)
    combo = [int(rng.integers(st.charges.shape[0])) for st in s0.sites]
    lam = np.concatenate([np.eye(st.charges.shape[0])[c] for st, c in zip(s0.sites, combo)])
    s = s0.with_lam(lam)
    E, F, _, _ = hi.hi_dense(s.q, s.sites, Phi, G)
    qx = brute.charges_of(s.q, s.sites, combo)
    assert abs(E - 0.5 * KE * qx @ Phi @ qx) <= 1e-12 * abs(E)
    assert rel(F, KE * qx[:, None] * np.einsum("ijk,j->ik", G, qx)) <= 1e-12


# ---------------------------------------------------------------- P5: Ewald constants

XI_SC = -2.837297479480620  # point charge in a neutralising background, simple cubic lattice


@pytest.mark.parametrize("alpha", [3.0, 5.0, 8.0])
def test_single_charge_self_energy(alpha):
    L = 2.5
    p, g = ewald.pair(np.zeros((1, 3)), L, alpha=alpha / L)
    assert abs(p[0] * L - XI_SC) <= 1e-12
    ph, E = ewald.field(np.array([[0.3, 1.7, 2.2]]), np.array([1.3]), L, alpha=alpha / L)
    assert abs(0.5 * 1.3 * ph[0] - 0.5 * 1.3 ** 2 * XI_SC / L) <= 1e-12
    assert np.abs(E).max() <= 1e-12


def _lattice(kind):
    if kind == "nacl":   # rock salt, conventional cube L = 1, nearest-neighbour distance 1/2
        x = np.array([[i, j, k] for i in (0, .5) for j in (0, .5) for k in (0, .5)], float)
        q = np.array([(-1.0) ** round(2 * (a + b + c)) for a, b, c in x])
        return x, q, -4 * 1.747564594633 / 0.5
    # caesium chloride, cube L = 1, nearest-neighbour distance sqrt(3)/2
    x = np.array([[0, 0, 0], [.5, .5, .5]], float)
    q = np.array([1.0, -1.0])
    return x, q, -1.762674773070 / (np.sqrt(3) / 2)


@pytest.mark.parametrize("kind", ["nacl", "cscl"])
@pytest.mark.parametrize("alpha", [2.0, 4.0, 7.0])
def test_madelung_constants(kind, alpha):
    x, q, ref = _lattice(kind)
    ph, E = ewald.field(x + 0.137, q, 1.0, alpha=alpha)
    assert abs(0.5 * q @ ph - ref) <= 1e-11 * abs(ref)
    assert np.abs(E).max() <= 1e-11   # every ion sits at a centre of symmetry


def test_pair_kernel_alpha_independent_and_periodic():
    rng = np.random.default_rng(2)
    L = 1.7
    r = rng.uniform(-L, L, (20, 3))
    p1, g1 = ewald.pair(r, L, alpha=2.5 / L)
    p2, g2 = ewald.pair(r, L, alpha=6.0 / L)
    p3, g3 = ewald.pair(r + L * np.array([1, -2, 3]), L, alpha=4.0 / L)
    assert np.abs(p1 - p2).max() <= 1e-12 * np.abs(p1).max()
    assert np.abs(g1 - g2).max() <= 1e-11 * np.abs(g1).max()
    assert np.abs(p1 - p3).max() <= 1e-12 * np.abs(p1).max()


def test_pair_kernel_gradient_by_finite_difference():
    rng = np.random.default_rng(3)
    L = 1.3
    r = rng.uniform(-L / 2, L / 2, (8, 3))
    _, g = ewald.pair(r, L)
    h = 1e-5
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        pp, _ = ewald.pair(r + e, L)
        pm, _ = ewald.pair(r - e, L)
        assert np.abs(-(pp - pm) / (2 * h) - g[:, d]).max() <= 1e-7 * np.abs(g).max()


def test_field_path_matches_pair_path():
    """Structure-factor Ewald (cell lists) equals the per-pair Ewald on a small periodic system."""
    s = small(True, n_w=40, edge=1.6)
    Phi, G = dense(s)
    E, F, dvdl, dedq = hi.hi_dense(s.q, s.sites, Phi, G)
    E2, F2, dvdl2, dedq2 = hi.hi_periodic(s.x, s.q, s.sites, s.box)
    assert abs(E - E2) <= 1e-12 * abs(E)
    assert rel(F2, F) <= 1e-12
    assert np.abs(dvdl2 - dvdl).max() <= 1e-11 * np.abs(dvdl).max()


# ---------------------------------------------------------------- open boundaries

def test_open_two_charges_analytic():
    x = np.array([[0.0, 0.0, 0.0], [0.3, 0.4, 0.0]])
    Phi, G = kernels.open_dense(x)
    q = np.array([1.0, -2.0])
    E, F, _, _ = hi.hi_dense(q, [], Phi, G)
    assert abs(E - KE * (-2.0 / 0.5)) <= 1e-12
    # attraction: atom 0 pulled towards atom 1
    assert np.allclose(F[0], KE * np.array([4.8, 6.4, 0.0]), rtol=1e-12, atol=0)
    assert np.allclose(F[1], -F[0], rtol=1e-12, atol=0)


# ---------------------------------------------------------------- P6, P7: invariants, finite differences

@pytest.mark.parametrize("periodic", [False, True])
def test_net_force_vanishes(periodic):
    s = small(periodic)
    Phi, G = dense(s)
    _, F, _, _ = hi.hi_dense(s.q, s.sites, Phi, G)
    assert np.abs(F.sum(0)).max() <= 1e-11 * np.abs(F).max()


def _energy(s):
    Phi, G = dense(s)
    return hi.hi_dense(s.q, s.sites, Phi, G)[0]


@pytest.mark.parametrize("periodic", [False, True])
def test_forces_by_central_difference(periodic):
    s = small(periodic)
    _, F, _, _ = hi.hi_dense(s.q, s.sites, *dense(s))
    h = 1e-5
    rng = np.random.default_rng(7)
    site_atoms = np.concatenate([st.atoms for st in s.sites])
    picks = list(site_atoms[:6]) + list(rng.integers(0, s.n_atoms, 4))
    for i in picks:
        for d in range(3):
            sp = System(s.name, s.periodic, s.box, s.x.astype(np.float64), s.q, s.sites)
            sm = System(s.name, s.periodic, s.box, s.x.astype(np.float64), s.q, s.sites)
            sp.x = sp.x.copy(); sm.x = sm.x.copy()
            sp.x[i, d] += h
            sm.x[i, d] -= h
            fd = -(_energy(sp) - _energy(sm)) / (2 * h)
            assert abs(fd - F[i, d]) <= 1e-6 * np.abs(F).max()


@pytest.mark.parametrize("periodic", [False, True])
def test_dvdl_by_central_difference_off_simplex(periodic):
    s = small(periodic)
    _, _, dvdl, _ = hi.hi_dense(s.q, s.sites, *dense(s))
    lam = s.lam_flat() * 0.9 + 0.03   # off the simplex on purpose
    s = s.with_lam(lam)
    _, _, dvdl, _ = hi.hi_dense(s.q, s.sites, *dense(s))
    h = 1e-4
    for k in range(lam.shape[0]):
        lp, lm = lam.copy(), lam.copy()
        lp[k] += h
        lm[k] -= h
        fd = (_energy(s.with_lam(lp)) - _energy(s.with_lam(lm))) / (2 * h)
        assert abs(fd - dvdl[k]) <= 1e-7 * np.abs(dvdl).max()


@pytest.mark.parametrize("periodic", [False, True])
def test_charge_derivative_by_central_difference(periodic):
    s = small(periodic)
    Phi, G = dense(s)
    _, _, _, dedq = hi.hi_dense(s.q, s.sites, Phi, G)
    h = 1e-4
    for si, st in enumerate(s.sites):
        for r in range(st.charges.shape[0]):
            for a in range(st.charges.shape[1]):
                vals = []
                for sgn in (1, -1):
                    sites = [Site(o.atoms, o.charges.copy(), o.lam) for o in s.sites]
                    sites[si].charges[r, a] += sgn * h
                    vals.append(hi.hi_dense(s.q, sites, Phi, G)[0])
                fd = (vals[0] - vals[1]) / (2 * h)
                assert abs(fd - dedq[si][r, a]) <= 1e-7 * max(abs(dedq[si]).max(), 1.0)


# ---------------------------------------------------------------- lambda transform (appendix)

def test_lambda_tilde_four_forms_as_printed():
    """Eq one_site_lambda: lt = ((1-l1)(1-l0), (1-l1) l0, l1 (1-l0), l1 l0)."""
    l0, l1 = 0.345, 0.721
    lt = lmap.lambda_tilde([l0, l1])
    ref = [(1 - l1) * (1 - l0), (1 - l1) * l0, l1 * (1 - l0), l1 * l0]
    assert np.allclose(lt, ref, rtol=0, atol=1e-15)
    assert abs(lt.sum() - 1.0) <= 1e-15


def test_mapping_table_matches_paper_with_reversed_bits():
    rows = np.loadtxt(os.path.join(HERE, "golden", "lambda_table.txt"), dtype=int)
    printed = rows[:, 1:].astype(bool)
    ours = lmap.mapping_table(3)
    # the printed table pairs lambda_0 with the most significant bit of rho
    rev = np.array([int(f"{r:03b}"[::-1], 2) for r in range(8)])
    assert np.array_equal(printed, ours[:, rev])


def test_back_map_equals_derivative_of_enumeration():
    """dH/dlambda_k from the chain rule equals the finite difference of the
    enumerated Hamiltonian of a 4-form site, at lambda = (0.345, 0.721)."""
    base = make_system(20, 1.4, False, [4], [4], total_step=None, depth=0, seed=21)
    Phi, G = dense(base)
    lams = np.array([0.345, 0.721])

    def H(ls):
        s = base.with_lam(lmap.lambda_tilde(ls))
        return brute.enumerate_hi(s.q, s.sites, Phi, G)[0]

    s = base.with_lam(lmap.lambda_tilde(lams))
    _, _, dvdl, _ = hi.hi_dense(s.q, s.sites, Phi, G)
    g = lmap.dlambda_from_dtilde(lams, dvdl)
    h = 1e-5
    for k in range(2):
        e = np.zeros(2)
        e[k] = h
        fd = (H(lams + e) - H(lams - e)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * np.abs(g).max()
    # two-form reference of eq ref_two_forms: dH/dlambda = H1 - H0
    b2 = make_system(20, 1.4, False, [4], [2], total_step=None, depth=0, seed=22)
    P2, G2 = dense(b2)
    s2 = b2.with_lam([0.655, 0.345])
    _, _, dv2, _ = hi.hi_dense(s2.q, s2.sites, P2, G2)
    H0 = brute.enumerate_hi(s2.q, s2.with_lam([1.0, 0.0]).sites, P2, G2)[0]
    H1 = brute.enumerate_hi(s2.q, s2.with_lam([0.0, 1.0]).sites, P2, G2)[0]
    assert abs((dv2[1] - dv2[0]) - (H1 - H0)) <= 1e-10 * abs(H1 - H0)


# ---------------------------------------------------------------- generators

def test_config_shapes_and_water_geometry():
    s = make_config(0)
    assert s.n_atoms == 1019 and len(s.sites) == 4 and s.n_forms == 8
    o, h1, h2 = s.x[0:999:3].astype(float), s.x[1:999:3].astype(float), s.x[2:999:3].astype(float)
    d1 = np.linalg.norm(h1 - o, axis=1)
    ang = np.degrees(np.arccos(np.einsum("ij,ij->i", h1 - o, h2 - o) / (d1 * np.linalg.norm(h2 - o, axis=1))))
    assert np.allclose(d1, 0.09572, atol=2e-6) and np.allclose(ang, 104.52, atol=1e-3)
    for st in s.sites:
        assert abs((st.charges[0].sum() - st.charges[1].sum()) - 1.0) <= 1e-12
        assert abs(st.lam.sum() - 1.0) <= 1e-15
    s1 = make_config(1)
    assert len(s1.sites) == 64 and s1.n_forms == 144
    assert (s1.x >= 0).all() and (s1.x < 10.0).all()
    assert np.array_equal(make_config(1).x, s1.x)
