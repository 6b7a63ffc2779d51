"""Measured launch-shape tuning (mahi_tune, run on an MI355X): the chosen M2L
operator ranges and near-field targets per lane are valid, change the results
only by rounding, and keep parity with the oracle's Ewald sums on the
100,717-atom system; argument and state errors are reported."""
import os

import numpy as np
import pytest

from synth import make_config, make_system

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_tune_float32_keeps_results_and_parity():
    import torch
    import paper_2410_01754_amd as pkg
    path = os.path.join(HERE, "golden", "config1_oracle.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    gd = np.load(path)
    s = make_config(1)
    print(f"[gpu] tune config1 N={s.n_atoms} p=8 d=4 prec=32", flush=True)
    m = pkg.from_system(s, precision=32, order=8, depth=4)
    before = m.eval(s.x)
    x = torch.from_numpy(s.x.astype(np.float32)).cuda()
    ranges, targets = m.tune(x.data_ptr(), reps=2)
    print(f"tuned: M2L operator ranges {ranges}, near-field targets per lane {targets}", flush=True)
    assert ranges in (1, 2, 3, 4, 5, 6, 8) and targets in (1, 2, 3)
    after = m.eval(s.x)
    again = m.eval(s.x)
    m.close()
    assert after["energy"] == again["energy"] and np.array_equal(after["forces"], again["forces"])
    assert abs(after["energy"] - before["energy"]) <= 1e-6 * abs(before["energy"])
    assert rel(after["forces"], before["forces"]) <= 1e-5
    assert rel(after["dvdl"], before["dvdl"]) <= 1e-5
    idx = gd["idx"]
    assert rel(after["forces"][idx], gd["forces"]) <= 2e-4
    assert rel(after["dvdl"], gd["dvdl"]) <= 2e-4


def test_tune_float64_and_errors():
    import torch
    import paper_2410_01754_amd as pkg
    from paper_2410_01754_amd.mahi import MahiError
    s = make_system(300, 2.2, True, [8, 8], [2, 3], total_step=1.0, depth=2, seed=11)
    print(f"[gpu] tune small N={s.n_atoms} p=8 d=2 prec=64", flush=True)
    m = pkg.from_system(s, precision=64, order=8, depth=2)
    x = torch.from_numpy(s.x.astype(np.float64)).cuda()
    before = m.eval(s.x)
    ranges, targets = m.tune(x.data_ptr(), reps=1)
    assert ranges == 0 and targets in (1, 2, 3)
    after = m.eval(s.x)
    assert rel(after["forces"], before["forces"]) <= 1e-12
    with pytest.raises(MahiError) as e:
        m.tune(x.data_ptr(), reps=0)
    assert "ERANGE" in str(e.value)
    m.close()
