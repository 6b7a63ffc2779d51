"""mahi_correct_noalloc (the correction with its scratch in a static device
array, for callers that cannot allocate) against mahi_correct (run on an
MI355X): same kernels, so the outputs must be bit-identical.  Two calls in a
row share the static array; the second has the smaller input.  Also: a
correction needing more scratch than the array holds is refused and writes
nothing; host-memory arguments are refused."""
import numpy as np
import pytest

from synth import Site, System, make_system

pytestmark = pytest.mark.gpu


def _system(n_waters, edge, big, seed):
    """Water box with clustered two- and three-form sites; `big` adds a 32-atom,
    16-form site, whose work arrays exceed local memory (the scratch then also
    holds the site pass's workspace)."""
    s = make_system(n_waters, edge, True, [6, 8, 5, 7], [2, 3, 2, 4], qrange=(-0.9, 0.9), total_step=None,
                    clustered=True, simplex=True, depth=2, seed=seed, name=f"noalloc{seed}")
    if not big:
        return s
    rng = np.random.default_rng(seed)
    n0 = s.n_atoms
    xb = (rng.random((32, 3)) * edge).astype(np.float32)
    site = Site(np.arange(n0, n0 + 32), rng.uniform(-0.9, 0.9, (16, 32)), rng.dirichlet(np.ones(16)))
    return System(s.name, True, s.box, np.concatenate([s.x, xb]), np.concatenate([s.q, np.zeros(32)]),
                  s.sites + [site], s.depth, 8, seed)


def _pair(s, precision):
    """mahi_correct and mahi_correct_noalloc on the tree's own potential of s."""
    import torch
    import paper_2410_01754_amd as pkg
    print(f"[gpu] {s.name} N={s.n_atoms} sites={len(s.sites)} prec={precision}", flush=True)
    dt = torch.float32 if precision == 32 else torch.float64
    m = pkg.from_system(s, precision=precision, order=8, depth=2)
    x = torch.from_numpy(s.x.astype(np.float32 if precision == 32 else np.float64)).cuda()
    pot = torch.zeros(s.n_atoms, dtype=dt, device="cuda")
    E0 = torch.zeros(1, dtype=torch.float64, device="cuda")
    F0 = torch.zeros((s.n_atoms, 3), dtype=dt, device="cuda")
    m.eval_device(x.data_ptr(), E0.data_ptr(), F0.data_ptr(), 0, pot.data_ptr())
    torch.cuda.synchronize()
    out = []
    for fn in (m.correct_device, m.correct_device_noalloc):
        E = torch.full((1,), 123.0, dtype=torch.float64, device="cuda")
        F = F0.clone()
        dv = torch.zeros(s.n_forms, dtype=torch.float64, device="cuda")
        dq = torch.zeros(m.n_form_charges, dtype=torch.float64, device="cuda")
        fn(x.data_ptr(), pot.data_ptr(), E.data_ptr(), F.data_ptr(), dv.data_ptr(), dq.data_ptr())
        torch.cuda.synchronize()
        out.append((E.cpu().numpy(), F.cpu().numpy(), dv.cpu().numpy(), dq.cpu().numpy()))
    m.close()
    return out


@pytest.mark.parametrize("precision", [32, 64])
def test_noalloc_matches_correct_twice(precision):
    for s in (_system(600, 2.6, True, 91), _system(250, 2.0, False, 92)):
        ref, got = _pair(s, precision)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
        assert ref[0][0] != 123.0


def test_noalloc_refuses_oversized_and_host_arguments():
    import torch
    import paper_2410_01754_amd as pkg
    rng = np.random.default_rng(93)
    # 80 sites of 32 atoms and 16 forms: 80 x 105 KB of work arrays > 8 MiB
    n = 80 * 32
    x = (rng.random((n, 3)) * 6.0).astype(np.float32)
    sites = [(np.arange(32 * k, 32 * k + 32), rng.uniform(-0.9, 0.9, (16, 32))) for k in range(80)]
    m = pkg.Mahi(6.0, True, np.zeros(n), sites, order=8, depth=2, precision=32)
    m.set_lambda(np.tile(np.full(16, 1.0 / 16), 80))
    xd = torch.from_numpy(x).cuda()
    pot = torch.zeros(n, dtype=torch.float32, device="cuda")
    E = torch.full((1,), 5.0, dtype=torch.float64, device="cuda")
    with pytest.raises(pkg.MahiError) as e:
        m.correct_device_noalloc(xd.data_ptr(), pot.data_ptr(), E.data_ptr())
    assert e.value.status == -4
    torch.cuda.synchronize()
    assert E.item() == 5.0
    # host memory is refused (the call only takes device pointers)
    from paper_2410_01754_amd.mahi import _CorrectArgs
    import ctypes
    Eh = np.zeros(1)
    args = _CorrectArgs(x.ctypes.data, np.zeros(n, np.float32).ctypes.data, Eh.ctypes.data, None, None, None, 0)
    assert m._lib.mahi_correct_noalloc(m._h, ctypes.byref(args)) == -1
    m.close()
