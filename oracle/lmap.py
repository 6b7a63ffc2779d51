"""lambda -> lambda-tilde transform and back-map of derivatives (oracle).

Appendix (eqs lambda_list, one_site_lambda and the index-tuple construction):
a site with 2^L forms is driven by L original lambdas; form rho gets the weight
  lt_rho = prod_k (lambda_k if bit k of rho is set else 1 - lambda_k).
Bit k of rho is matched to lambda_k with the least significant bit first, as in
eq one_site_lambda (rho = 1 <-> (1 - lambda_1) lambda_0).  The table of the
correction mapping prints lambda_0 against the most significant bit; that table
is read here as the same mapping with the bit order reversed.

Chain rule: with the derivatives g_rho = dH/dlt_rho,
  dH/dlambda_k = sum_rho s(rho,k) f(rho,k) g_rho,
where s = +1 if bit k is set and -1 otherwise, and f(rho,k) is the product of
the other L-1 factors of lt_rho.
"""
from __future__ import annotations

import numpy as np


def lambda_tilde(lams) -> np.ndarray:
    lams = np.asarray(lams, dtype=np.float64)
    L = lams.shape[0]
    out = np.ones(1 << L)
    for rho in range(1 << L):
        for k in range(L):
            out[rho] *= lams[k] if (rho >> k) & 1 else 1.0 - lams[k]
    return out


def dlambda_from_dtilde(lams, g) -> np.ndarray:
    lams = np.asarray(lams, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    L = lams.shape[0]
    out = np.zeros(L)
    for k in range(L):
        for rho in range(1 << L):
            f = 1.0
            for l in range(L):
                if l != k:
                    f *= lams[l] if (rho >> l) & 1 else 1.0 - lams[l]
            out[k] += (1.0 if (rho >> k) & 1 else -1.0) * f * g[rho]
    return out


def mapping_table(L: int) -> np.ndarray:
    """Boolean [2L, 2^L]: row 2k+b marks the forms whose bit k equals b."""
    t = np.zeros((2 * L, 1 << L), dtype=bool)
    for k in range(L):
        for rho in range(1 << L):
            t[2 * k + ((rho >> k) & 1), rho] = True
    return t
