"""Accuracy of the lambda forces against separately computed Hamiltonians (run on an MI355X).

The paper's random-system accuracy test (section "Random Systems" of the
methods, results in the section on the accuracy of the two- and four-form
random systems): 1,000 background particles and one 10-atom site, charges
uniform in [-1, 1], a clustered site ("typical") and a site spread over the
whole box ("worst case"), two forms (lambda = 0.345) and four forms of a
binary site (lambda = (0.345, 0.721)).  The reference lambda forces come from
one plain FMM run per form, at the same order and depth, without sites:
with H_X the energy of the system in form X, dE/dlambda-tilde_X differs from
H_X by the X-independent background energy, so the reference is
F_ref = -dlambda(lambda, H) with the same lambda -> lambda-tilde mapping as the
MAHI forces F = -dlambda(lambda, dE/dlambda-tilde).

What the paper fixes, and is asserted here:
* depth 0 (every interaction direct): F equals F_ref to rounding;
* depth > 0 in float64: the deviation comes from multipole truncation only,
  so it falls with the order, and the clustered site deviates far less than
  the spread one;
* in float32 the deviation sits at the single-precision level whatever the
  order (bounded here at depth 0 only).
The full table is printed.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

L_BOX = 4.0
LAMBDAS = {2: [0.345], 4: [0.345, 0.721]}
_FLOAT64_TABLES = {}  # (layout, n_forms) -> {(depth, order): deviation}


def x1_system(layout, n_forms, seed=1010):
    rng = np.random.default_rng(seed)
    x_env = rng.random((1000, 3)) * L_BOX
    if layout == "typical":
        c = rng.random(3) * L_BOX
        d = rng.normal(size=(10, 3))
        d *= (0.3 * rng.random(10) ** (1 / 3) / np.linalg.norm(d, axis=1))[:, None]
        x_site = np.mod(c + d, L_BOX)
    else:
        x_site = rng.random((10, 3)) * L_BOX
    q = np.concatenate([rng.uniform(-1, 1, 1000), np.zeros(10)])
    qf = rng.uniform(-1, 1, (n_forms, 10))
    return np.concatenate([x_env, x_site]), q, qf


def deviation(layout, n_forms, prec, order, depth):
    import paper_2410_01754_amd as pkg
    print(f"[gpu] x1 {layout} forms={n_forms} prec={prec} p={order} d={depth}", flush=True)
    x, q, qf = x1_system(layout, n_forms)
    lam = LAMBDAS[n_forms]
    xs = x.astype(np.float32 if prec == 32 else np.float64)
    m = pkg.Mahi(L_BOX, True, q, [(np.arange(1000, 1010), qf)], order=order, depth=depth, precision=prec)
    m.set_lambda(pkg.lambda_tilde(lam))
    F = -pkg.dlambda(lam, m.eval(xs, forces=False)["dvdl"])
    m.close()
    H = np.zeros(n_forms)
    for f in range(n_forms):
        qx = q.copy()
        qx[1000:] = qf[f]
        r = pkg.Mahi(L_BOX, True, qx, [], order=order, depth=depth, precision=prec)
        H[f] = r.eval(xs, forces=False)["energy"]
        r.close()
    Fref = -pkg.dlambda(lam, H)
    return float(np.max(np.abs(F - Fref) / np.abs(Fref)))


@pytest.mark.parametrize("n_forms", [2, 4])
@pytest.mark.parametrize("layout", ["typical", "worst"])
def test_x1_float64(layout, n_forms):
    tab = {}
    for d in (0, 2, 3):
        for p in (4, 8, 12):
            tab[d, p] = deviation(layout, n_forms, 64, p, d)
    print(layout, n_forms, "float64", {k: f"{v:.1e}" for k, v in tab.items()})
    for p in (4, 8, 12):
        assert tab[0, p] <= 1e-11
    for d in (2, 3):
        assert tab[d, 12] < tab[d, 4]
        assert tab[d, 12] <= 1e-6  # order-12 truncation of a handful of far site pairs
    _FLOAT64_TABLES[layout, n_forms] = tab


@pytest.mark.parametrize("n_forms", [2, 4])
@pytest.mark.parametrize("layout", ["typical", "worst"])
def test_x1_float32(layout, n_forms):
    tab = {}
    for d in (0, 2, 3):
        for p in (4, 8):
            tab[d, p] = deviation(layout, n_forms, 32, p, d)
    print(layout, n_forms, "float32", {k: f"{v:.1e}" for k, v in tab.items()})
    for p in (4, 8):
        assert tab[0, p] <= 1e-3


def test_x1_clustered_site_deviates_less():
    """At the lowest order, where truncation dominates, the spread site deviates more."""
    if len(_FLOAT64_TABLES) < 4:
        pytest.skip("needs the float64 sweeps of this module")
    for n_forms in (2, 4):
        for d in (2, 3):
            assert _FLOAT64_TABLES["typical", n_forms][d, 4] <= _FLOAT64_TABLES["worst", n_forms][d, 4]
