"""Invariances of the HIP path and the order of its calls (run on an MI355X).

* Permuting the atom order permutes the outputs and changes nothing else beyond
  rounding (the octree sorts atoms by position; within a leaf by index, so a
  permutation only reorders sums).
* Relabelling the forms of a site (with their weights) permutes that site's
  dE/dlambda-tilde; energy and forces are unchanged beyond rounding.  The
  general formulation (Theory, eq iter_ham_lambda) is a sum over forms, so its
  value cannot depend on their labels.
* mahi_eval before mahi_set_lambda returns MAHI_ESTATE and writes nothing.
"""
import ctypes

import numpy as np
import pytest

from synth import Site, System, make_system

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run(s, precision, order, depth):
    import paper_2410_01754_amd as pkg
    print(f"[gpu] {s.name} N={s.n_atoms} p={order} d={depth} prec={precision}", flush=True)
    m = pkg.from_system(s, precision=precision, order=order, depth=depth)
    out = m.eval(s.x, dedq=True)
    m.close()
    return out


def base_system(seed):
    return make_system(400, 2.4, True, [6, 8, 5, 7], [2, 3, 2, 4], qrange=(-0.9, 0.9), total_step=None,
                       clustered=True, simplex=True, depth=2, seed=seed, name="invariance")


# rounding bounds: float64 sums reordered (1e-12); float32 sums reordered over
# ~700 near-field terms and an order-8 local expansion (1e-5)
TOL = {64: 1e-12, 32: 1e-5}


@pytest.mark.parametrize("prec", [64, 32])
def test_atom_permutation_changes_only_rounding(prec):
    s = base_system(61)
    rng = np.random.default_rng(62)
    perm = rng.permutation(s.n_atoms)  # new atom k is old atom perm[k]
    inv = np.empty_like(perm)
    inv[perm] = np.arange(s.n_atoms)
    sites = [Site(inv[st.atoms], st.charges.copy(), st.lam.copy()) for st in s.sites]
    sp = System(s.name, True, s.box, s.x[perm].copy(), s.q[perm].copy(), sites, s.depth, 8, s.seed)
    a, b = run(s, prec, 8, 2), run(sp, prec, 8, 2)
    tol = TOL[prec]
    assert abs(b["energy"] - a["energy"]) <= tol * abs(a["energy"])
    assert rel(b["forces"], a["forces"][perm]) <= tol
    assert rel(b["dvdl"], a["dvdl"]) <= tol
    assert rel(b["dedq"], a["dedq"]) <= tol


@pytest.mark.parametrize("prec", [64, 32])
def test_form_relabelling_permutes_dvdl(prec):
    s = base_system(63)
    rng = np.random.default_rng(64)
    sites, order, dq_order, o, fo = [], [], [], 0, 0
    for st in s.sites:
        nf, na = st.charges.shape
        pf = rng.permutation(nf)  # new form r is old form pf[r]
        sites.append(Site(st.atoms.copy(), st.charges[pf].copy(), st.lam[pf].copy()))
        order.extend(o + pf)
        dq_order.extend((fo + pf[:, None] * na + np.arange(na)[None, :]).reshape(-1))
        o += nf
        fo += nf * na
    sp = System(s.name, True, s.box, s.x, s.q, sites, s.depth, 8, s.seed)
    a, b = run(s, prec, 8, 2), run(sp, prec, 8, 2)
    tol = TOL[prec]
    assert abs(b["energy"] - a["energy"]) <= tol * abs(a["energy"])
    assert rel(b["forces"], a["forces"]) <= tol
    assert rel(b["dvdl"], a["dvdl"][np.array(order)]) <= tol
    assert rel(b["dedq"], a["dedq"][np.array(dq_order)]) <= tol


def test_eval_before_set_lambda_is_refused():
    import paper_2410_01754_amd as pkg
    from paper_2410_01754_amd.mahi import _EvalArgs
    s = base_system(65)
    sites = [(st.atoms, st.charges) for st in s.sites]
    m = pkg.Mahi(s.box, True, s.q, sites, order=8, depth=2, precision=32)
    x = np.ascontiguousarray(s.x, dtype=np.float32)
    E = np.full(1, 12345.0)
    F = np.full((s.n_atoms, 3), 7.0, dtype=np.float32)
    dv = np.full(m.n_forms, -3.0)
    args = _EvalArgs(x.ctypes.data, E.ctypes.data, F.ctypes.data, dv.ctypes.data, None, 0, None, None, None)
    st = m._lib.mahi_eval(m._h, ctypes.byref(args))
    assert st == -5  # MAHI_ESTATE
    assert E[0] == 12345.0 and np.all(F == 7.0) and np.all(dv == -3.0)
    # after mahi_set_lambda the same call succeeds and writes the outputs
    m.set_lambda(s.lam_flat())
    assert m._lib.mahi_eval(m._h, ctypes.byref(args)) == 0
    assert E[0] != 12345.0 and not np.all(F == 7.0)
    m.close()
