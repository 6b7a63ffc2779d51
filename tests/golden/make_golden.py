"""Write oracle reference values for the large seeded configurations.

Calls only oracle/ and synth/ (never the GPU library).  Output per config:
tests/golden/config<k>_oracle.npz with the HI energy, dE/dlambda-tilde of
every form, dE/dq of every form charge, the charge-interpolation energy and
its dE/dlambda-tilde, and forces at every site atom plus a seeded sample of
other atoms.

Usage: [ORACLE_THREADS=n] python tests/golden/make_golden.py 1 [2]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import hi  # noqa: E402
from synth import make_config  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def sample_atoms(system, n_env=4000, seed=99):
    rng = np.random.default_rng(seed)
    site = np.concatenate([s.atoms for s in system.sites])
    env = rng.choice(system.n_atoms - site.shape[0], size=min(n_env, system.n_atoms - site.shape[0]), replace=False)
    return np.unique(np.concatenate([site, env]))


def main(k):
    s = make_config(k)
    t = time.time()
    idx = sample_atoms(s)
    nthreads = int(os.environ.get("ORACLE_THREADS", "0"))  # 0: every host core
    E, F, dvdl, dedq, E_qi, dvdl_qi = hi.hi_periodic(s.x, s.q, s.sites, s.box, qi=True, nthreads=nthreads)
    dt = time.time() - t
    out = os.path.join(HERE, f"config{k}_oracle.npz")
    np.savez_compressed(out, energy=np.array([E]), dvdl=dvdl, idx=idx, forces=F[idx],
                        force_norm=np.array([np.linalg.norm(F)]), seconds=np.array([dt]),
                        dedq=np.concatenate([d.reshape(-1) for d in dedq]), energy_qi=np.array([E_qi]),
                        dvdl_qi=dvdl_qi)
    print(f"config{k}: N={s.n_atoms} E={E:.10f} oracle {dt:.1f}s -> {out}", flush=True)


if __name__ == "__main__":
    for a in sys.argv[1:]:
        main(int(a))
