"""Brute-force HI by enumeration of every site-form combination (oracle, tiny N).

The interpolated Hamiltonian is the weighted sum of sub-Hamiltonians, one per
combination X of forms (eq rek_ham_lambda, generalised to any number of sites
and forms in the appendix): H = sum_X (prod_sigma lt_{sigma, X_sigma}) H_X with
H_X = 1/2 q_X . Phi . q_X (eq nbody_periodic; Phi's diagonal holds the self
images of a periodic cube, zero for open boundaries).  The HI force is the same
weighted sum of the fixed-charge forces, and dH/dq^(sigma,rho)_i sums the
potentials of the combinations that put site sigma in form rho.
"""
from __future__ import annotations

import itertools

import numpy as np

from .hi import KE_DEFAULT


def charges_of(q, sites, combo):
    qx = np.array(q, dtype=np.float64, copy=True)
    for st, r in zip(sites, combo):
        qx[st.atoms] = st.charges[r]
    return qx


def enumerate_hi(q, sites, Phi, G, ke=KE_DEFAULT):
    """E, F and dE/dq by explicit enumeration (cost prod(#forms) dense products)."""
    E = 0.0
    F = np.zeros((Phi.shape[0], 3))
    dedq = [np.zeros_like(st.charges) for st in sites]
    for combo in itertools.product(*[range(st.charges.shape[0]) for st in sites]):
        w = 1.0
        for st, r in zip(sites, combo):
            w *= st.lam[r]
        qx = charges_of(q, sites, combo)
        V = Phi @ qx
        E += w * 0.5 * qx @ V
        F += w * qx[:, None] * np.einsum("ijk,j->ik", G, qx)
        for s, (st, r) in enumerate(zip(sites, combo)):
            dedq[s][r] += w * V[st.atoms]
    return ke * E, ke * F, [ke * d for d in dedq]


def dvdl_by_deletion(q, sites, Phi, ke=KE_DEFAULT):
    """dH/dlt_(sigma,rho) = H(site sigma fixed to form rho) - H(site sigma removed).

    H is affine in the weights of one site, so the difference of its values at
    the vertex e_rho and at the origin (zero charges, no form-form term) is the
    partial derivative.  Both values are brute-force enumerations over the other
    sites, with site sigma's charges fixed or zeroed.
    """
    out = []
    for s, st in enumerate(sites):
        others = [o for k, o in enumerate(sites) if k != s]
        q0 = np.array(q, dtype=np.float64, copy=True)
        q0[st.atoms] = 0.0
        e_del = enumerate_hi(q0, others, Phi, np.zeros(Phi.shape + (3,)), ke)[0]
        for r in range(st.charges.shape[0]):
            qr = q0.copy()
            qr[st.atoms] = st.charges[r]
            out.append(enumerate_hi(qr, others, Phi, np.zeros(Phi.shape + (3,)), ke)[0] - e_del)
    return np.array(out)
