"""HI energy and derivatives from the paper's general formulation (oracle).

General formulation (Theory, eq iter_ham_lambda, with the box shifts of eq
nbody_periodic): with lambda-tilde scaled charges qt_i = sum_rho lt_rho q^rho_i
at site atoms (eq after eq constraint) and qt_i = q_i in the environment,

  H = 1/2 sum_{i,j not in the same site} qt_i qt_j Phi_ij
      + sum_sigma sum_rho lt^(sigma,rho) 1/2 sum_{i,j in sigma} q^rho_i q^rho_j Phi_ij .

The first sum is env-env + env-site + site-site; the second is form-form.
Derivatives are taken of this expression with every lambda-tilde treated as an
independent variable (it is affine in the weights of each site):

  Vext_i      = sum_{j not in the site of i} qt_j Phi_ij
  dH/dlt_srho = sum_{i in s} q^rho_i Vext_i + 1/2 q^rho . Phi_ss . q^rho
  F_i         = qt_i sum_{j not in the site of i} qt_j G_ij
                + [i in s] sum_rho lt_rho q^rho_i sum_{j in s} q^rho_j G_ij
  dH/dq^srho_i = lt_rho (Vext_i + sum_{j in s} Phi_ij q^rho_j)

All outputs are multiplied by the Coulomb constant ke (kJ mol^-1 nm e^-2 by
default).  Periodic systems use Ewald sums; open ones the direct sum.
"""
from __future__ import annotations

import numpy as np

from . import ewald, kernels

KE_DEFAULT = 138.9354576


def scaled_charges(n, q, sites):
    qt = np.array(q, dtype=np.float64, copy=True)
    site_of = -np.ones(n, dtype=np.int64)
    for s, st in enumerate(sites):
        qt[st.atoms] = st.lam @ st.charges
        site_of[st.atoms] = s
    return qt, site_of


def hi_dense(q, sites, Phi, G, ke=KE_DEFAULT):
    """HI outputs from dense Phi [N,N] and G [N,N,3] (small systems)."""
    n = Phi.shape[0]
    qt, site_of = scaled_charges(n, q, sites)
    same = (site_of[:, None] == site_of[None, :]) & (site_of[:, None] >= 0)
    Pext = np.where(same, 0.0, Phi)
    Vext = Pext @ qt
    fext = np.einsum("ijk,j->ik", np.where(same[:, :, None], 0.0, G), qt)
    E = 0.5 * qt @ Vext
    F = qt[:, None] * fext
    dvdl, dedq = [], []
    for st in sites:
        a = st.atoms
        Pss = Phi[np.ix_(a, a)]
        Gss = G[np.ix_(a, a)]
        dq = np.zeros_like(st.charges)
        for r in range(st.charges.shape[0]):
            qr = st.charges[r]
            self_r = 0.5 * qr @ Pss @ qr
            E += st.lam[r] * self_r
            dvdl.append(qr @ Vext[a] + self_r)
            F[a] += st.lam[r] * qr[:, None] * np.einsum("ijk,j->ik", Gss, qr)
            dq[r] = st.lam[r] * (Vext[a] + Pss @ qr)
        dedq.append(ke * dq)
    return ke * E, ke * F, ke * np.array(dvdl), dedq


def hi_periodic(x, q, sites, L, ke=KE_DEFAULT, targets=None, nthreads=0, alpha=None, qi=False):
    """HI outputs for a periodic cube via Ewald sums.

    Returns E, F, dvdl, dedq.  With `targets` given, F is returned only for
    those atoms and E is None (the energy needs the potential at every atom).
    With qi=True two more values follow, the charge-interpolation outputs of
    qi_dense from the same field: E_QI (None with `targets`) and dvdl_QI.
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    qt, site_of = scaled_charges(n, q, sites)
    site_atoms = np.concatenate([st.atoms for st in sites]) if sites else np.zeros(0, dtype=np.int64)
    if targets is None:
        tg = np.arange(n)
    else:
        tg = np.unique(np.concatenate([np.asarray(targets, dtype=np.int64), site_atoms]))
    phi, fld = ewald.field(x, qt, L, targets=tg, alpha=alpha, nthreads=nthreads)
    pos = {int(t): k for k, t in enumerate(tg)}
    Vext = phi.copy()
    fext = fld.copy()
    blocks = []
    for st in sites:
        a = st.atoms
        d = (x[a][:, None, :] - x[a][None, :, :]).reshape(-1, 3)
        pp, gg = ewald.pair(d, L)
        Pss = pp.reshape(len(a), len(a))
        Gss = gg.reshape(len(a), len(a), 3)
        ia = np.array([pos[int(i)] for i in a])
        Vext[ia] -= Pss @ qt[a]
        fext[ia] -= np.einsum("ijk,j->ik", Gss, qt[a])
        blocks.append((ia, Pss, Gss))
    F = qt[tg][:, None] * fext
    E = 0.5 * qt[tg] @ Vext if targets is None else None
    dvdl, dedq = [], []
    for st, (ia, Pss, Gss) in zip(sites, blocks):
        dq = np.zeros_like(st.charges)
        for r in range(st.charges.shape[0]):
            qr = st.charges[r]
            self_r = 0.5 * qr @ Pss @ qr
            if E is not None:
                E += st.lam[r] * self_r
            dvdl.append(qr @ Vext[ia] + self_r)
            F[ia] += st.lam[r] * qr[:, None] * np.einsum("ijk,j->ik", Gss, qr)
            dq[r] = st.lam[r] * (Vext[ia] + Pss @ qr)
        dedq.append(ke * dq)
    Eo = None if E is None else ke * E
    out = (Eo, ke * F, ke * np.array(dvdl), dedq) if targets is None else (Eo, (tg, ke * F), ke * np.array(dvdl), dedq)
    if not qi:
        return out
    # phi is the full scaled-charge potential (before the site blocks were removed)
    dv_qi = [st.charges[r] @ phi[ia] for st, (ia, _, _) in zip(sites, blocks) for r in range(st.charges.shape[0])]
    E_qi = ke * 0.5 * qt[tg] @ phi if targets is None else None
    return out + (E_qi, ke * np.array(dv_qi))


def qi_dense(q, sites, Phi, ke=KE_DEFAULT):
    """Charge interpolation (section "Comparison of Hamiltonian and Charge
    Interpolation"): the scaled charges treated as fixed charges,
      E_QI = 1/2 qt.Phi.qt,   dE_QI/dlt_srho = sum_{i in s} q^rho_i (Phi qt)_i
    (chain rule through qt_i = sum_rho lt_rho q^rho_i).  Returns E_QI, dvdl_QI."""
    qt, _ = scaled_charges(Phi.shape[0], q, sites)
    V = Phi @ qt
    dv = [st.charges[r] @ V[st.atoms] for st in sites for r in range(st.charges.shape[0])]
    return ke * 0.5 * qt @ V, ke * np.array(dv)


def qi_periodic(x, q, sites, L, ke=KE_DEFAULT, nthreads=0, alpha=None):
    """qi_dense for a periodic cube: Phi qt from the Ewald field at every atom."""
    x = np.asarray(x, dtype=np.float64)
    qt, _ = scaled_charges(x.shape[0], q, sites)
    V, _ = ewald.field(x, qt, L, alpha=alpha, nthreads=nthreads)
    dv = [st.charges[r] @ V[st.atoms] for st in sites for r in range(st.charges.shape[0])]
    return ke * 0.5 * qt @ V, ke * np.array(dv)


def evaluate(system, ke=KE_DEFAULT, dense_limit=3000, nthreads=0):
    """Dispatch on boundary type and size; returns E, F, dvdl, dedq."""
    if not system.periodic:
        Phi, G = kernels.open_dense(system.x)
        return hi_dense(system.q, system.sites, Phi, G, ke)
    if system.n_atoms <= dense_limit // 10:
        Phi, G = kernels.periodic_dense(system.x, system.box)
        return hi_dense(system.q, system.sites, Phi, G, ke)
    return hi_periodic(system.x, system.q, system.sites, system.box, ke, nthreads=nthreads)
