"""Batched evaluation of many small systems and the autotuner (run on an MI355X).

* A batch (eager fork/join; its captured-graph mode is refused and its case
  skipped) gives the same bits as evaluating each system alone, repeatedly,
  after a change of lambda-tilde and with new output buffers.
* A packed batch (every stage one launch over all systems) agrees with the
  single evaluations up to float32 rounding; its HIP-graph replays equal its
  eager calls bit for bit.
* Systems evaluated with the autotuned order and depth meet the accuracy
  target against the oracle's Ewald sums.
"""
import numpy as np
import pytest

from oracle import hi
from synth import make_batch

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _build(systems, precision=32, target=2e-4):
    import paper_2410_01754_amd as pkg
    mods = []
    for s in systems:
        p, d = pkg.autotune(True, s.box, s.n_atoms, precision, target, pkg.site_extent(s))
        print(f"[gpu] {s.name} N={s.n_atoms} p={p} d={d} prec={precision}", flush=True)
        mods.append(pkg.from_system(s, precision=precision, order=p, depth=d))
    return mods


def _buffers(systems, dtype):
    import torch
    out = []
    for s in systems:
        out.append({"x": torch.from_numpy(s.x.astype(np.float32 if dtype == torch.float32 else np.float64)).cuda(),
                    "E": torch.zeros(1, dtype=torch.float64, device="cuda"),
                    "F": torch.zeros((s.n_atoms, 3), dtype=dtype, device="cuda"),
                    "dv": torch.zeros(s.n_forms, dtype=torch.float64, device="cuda")})
    return out


def _ptrs(bufs):
    return [{"xyz": b["x"].data_ptr(), "energy": b["E"].data_ptr(), "forces": b["F"].data_ptr(),
             "dvdl": b["dv"].data_ptr()} for b in bufs]


def _same(bufs, refs):
    for b, r in zip(bufs, refs):
        assert b["E"].item() == r["energy"]
        assert np.array_equal(b["F"].cpu().numpy(), r["forces"])
        assert np.array_equal(b["dv"].cpu().numpy(), r["dvdl"])


@pytest.mark.parametrize("use_graph", [False, pytest.param(True, marks=pytest.mark.skip(
    reason="graph capture of a batch is disabled: its first capture and launch ended in a host segmentation "
           "fault whose cause is not yet shown"))])
def test_batch_matches_single_evaluations(use_graph):
    import torch
    import paper_2410_01754_amd as pkg
    systems = make_batch(n_systems=6, n_min=1500, n_max=8000, seed=77)
    mods = _build(systems)
    refs = [m.eval(s.x) for m, s in zip(mods, systems)]
    bufs = _buffers(systems, torch.float32)
    batch = pkg.Batch(mods, use_graph=use_graph)
    for rep in range(3):
        for b in bufs:
            b["E"].zero_()
            b["F"].zero_()
            b["dv"].zero_()
        torch.cuda.synchronize()
        batch.eval_device(_ptrs(bufs))
        torch.cuda.synchronize()
        print(f"[gpu] batch graph={use_graph} replay {rep}", flush=True)
        _same(bufs, refs)
        # eager work between replays
        torch.cuda.synchronize()
        _ = (bufs[0]["F"] * 2.0).sum().item()
    # new weights for system 0: a replay reads them from device memory
    lam = systems[0].lam_flat().copy()
    lam[0::2], lam[1::2] = lam[1::2].copy(), lam[0::2].copy()
    mods[0].set_lambda(lam)
    refs[0] = mods[0].eval(systems[0].x)
    batch.eval_device(_ptrs(bufs))
    torch.cuda.synchronize()
    _same(bufs, refs)
    # new output buffers: the batch captures again
    bufs2 = _buffers(systems, torch.float32)
    batch.eval_device(_ptrs(bufs2))
    torch.cuda.synchronize()
    _same(bufs2, refs)
    batch.close()
    for m in mods:
        m.close()


def _fresh(bufs):
    for b in bufs:
        b["E"].zero_()
        b["F"].zero_()
        b["dv"].zero_()


def _close(bufs, refs, tol):
    for b, r in zip(bufs, refs):
        e = abs(b["E"].item() - r["energy"]) / abs(r["energy"])
        f = rel(b["F"].cpu().numpy(), r["forces"])
        v = rel(b["dv"].cpu().numpy(), r["dvdl"])
        assert e <= tol and f <= tol and v <= tol, (e, f, v)


def test_packed_batch_matches_single_evaluations():
    """Packed batch (every stage one launch over all systems, systems of depth
    2..4): the same arithmetic as evaluating each system alone except the
    summation order of the M2L operator ranges (float32 rounding), and the
    oracle's accuracy bound; repeated calls are bit-identical."""
    import torch
    import paper_2410_01754_amd as pkg
    systems = make_batch(n_systems=7, n_min=1500, n_max=30000, seed=80)
    mods = _build(systems)
    refs = [m.eval(s.x) for m, s in zip(mods, systems)]
    bufs = _buffers(systems, torch.float32)
    batch = pkg.Batch(mods, packed=True)
    outs = []
    for rep in range(2):
        _fresh(bufs)
        torch.cuda.synchronize()
        batch.eval_device(_ptrs(bufs))
        torch.cuda.synchronize()
        print(f"[gpu] packed batch call {rep}", flush=True)
        _close(bufs, refs, 1e-5)
        outs.append([(b["E"].item(), b["F"].cpu().numpy(), b["dv"].cpu().numpy()) for b in bufs])
    for a, b in zip(outs[0], outs[1]):
        assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    # new weights of one system are read at the next call
    lam = systems[1].lam_flat().copy()
    lam[0::2], lam[1::2] = lam[1::2].copy(), lam[0::2].copy()
    mods[1].set_lambda(lam)
    refs[1] = mods[1].eval(systems[1].x)
    batch.eval_device(_ptrs(bufs))
    torch.cuda.synchronize()
    _close(bufs, refs, 1e-5)
    s = systems[0]
    E, F, dv, _ = hi.hi_periodic(s.x, s.q, s.sites, s.box)
    assert rel(bufs[0]["F"].cpu().numpy(), F) <= 2e-4 and rel(bufs[0]["dv"].cpu().numpy(), dv) <= 2e-4
    batch.close()
    for m in mods:
        m.close()


def test_packed_batch_high_order():
    """Spread sites get order 9 from the autotuner: the packed batch then runs the
    32x32x2 M2L kernel; it agrees with single evaluations up to rounding."""
    import torch
    import paper_2410_01754_amd as pkg
    from synth import make_system
    rng = np.random.default_rng(84)
    systems = [make_system(int(n / 3), (n / 3 / 33.4) ** (1 / 3), True, [8] * 5, [2] * 5, total_step=None,
                           clustered=False, seed=int(rng.integers(1 << 30)), name=f"hi{k}")
               for k, n in enumerate((2500, 9000, 20000))]
    mods = _build(systems)
    assert all(m.info()["order"] == 9 for m in mods)
    refs = [m.eval(s.x) for m, s in zip(mods, systems)]
    bufs = _buffers(systems, torch.float32)
    batch = pkg.Batch(mods, packed=True)
    batch.eval_device(_ptrs(bufs))
    torch.cuda.synchronize()
    _close(bufs, refs, 1e-5)
    batch.close()
    for m in mods:
        m.close()


def test_packed_batch_graph_replays():
    """The packed launches captured in a HIP graph: every replay equals the eager
    packed call bit for bit, with eager work and synchronisations between
    replays, after new weights, and after new output buffers (a new capture)."""
    import torch
    import paper_2410_01754_amd as pkg
    systems = make_batch(n_systems=5, n_min=1500, n_max=12000, seed=81)
    mods = _build(systems)
    bufs = _buffers(systems, torch.float32)
    eager = pkg.Batch(mods, packed=True)
    eager.eval_device(_ptrs(bufs))
    torch.cuda.synchronize()
    ref = [(b["E"].item(), b["F"].cpu().numpy(), b["dv"].cpu().numpy()) for b in bufs]
    graph = pkg.Batch(mods, packed=True, use_graph=True)

    def same(bs, rs):
        for b, r in zip(bs, rs):
            assert b["E"].item() == r[0]
            assert np.array_equal(b["F"].cpu().numpy(), r[1]) and np.array_equal(b["dv"].cpu().numpy(), r[2])

    for rep in range(3):
        _fresh(bufs)
        torch.cuda.synchronize()
        graph.eval_device(_ptrs(bufs))
        torch.cuda.synchronize()
        print(f"[gpu] packed graph replay {rep}", flush=True)
        same(bufs, ref)
        _ = (bufs[0]["F"] * 2.0).sum().item()
    lam = systems[2].lam_flat().copy()
    lam[0::2], lam[1::2] = lam[1::2].copy(), lam[0::2].copy()
    mods[2].set_lambda(lam)
    eager.eval_device(_ptrs(bufs))
    torch.cuda.synchronize()
    ref = [(b["E"].item(), b["F"].cpu().numpy(), b["dv"].cpu().numpy()) for b in bufs]
    _fresh(bufs)
    graph.eval_device(_ptrs(bufs))
    torch.cuda.synchronize()
    same(bufs, ref)
    bufs2 = _buffers(systems, torch.float32)
    graph.eval_device(_ptrs(bufs2))
    torch.cuda.synchronize()
    same(bufs2, ref)
    graph.close()
    eager.close()
    for m in mods:
        m.close()


def _tangent(dv, s):
    out, o = [], 0
    for st in s.sites:
        nf = st.charges.shape[0]
        out.extend(dv[o + r] - dv[o] for r in range(1, nf))
        o += nf
    return np.array(out)


@pytest.mark.parametrize("clustered", [True, False])
def test_autotuned_systems_meet_target(clustered):
    """Systems of 3k..60k atoms with clustered or spread two-form sites, each with
    the autotuned order and depth for 2e-4: energy, forces and dE/dlambda-tilde
    within the target against the oracle; the tangent (the lambda forces, an
    RMS over only 4..16 sites here) within twice the target."""
    from synth import make_system
    rng = np.random.default_rng(82 if clustered else 83)
    systems = []
    for k, n_tot in enumerate((3000, 14000, 60000)):
        n_s = int(rng.integers(4, 16))
        n_w = (n_tot - 8 * n_s) // 3
        edge = (n_w / 33.4) ** (1 / 3)
        systems.append(make_system(n_w, edge, True, [8] * n_s, [2] * n_s, total_step=None, clustered=clustered,
                                   seed=int(rng.integers(1 << 30)), name=f"tuned{k}"))
    mods = _build(systems, precision=32, target=2e-4)
    for m, s in zip(mods, systems):
        g = m.eval(s.x)
        E, F, dv, _ = hi.hi_periodic(s.x, s.q, s.sites, s.box)
        e = (abs(g["energy"] - E) / abs(E), rel(g["forces"], F), rel(g["dvdl"], dv),
             rel(_tangent(g["dvdl"], s), _tangent(dv, s)))
        print(f"{s.name} N={s.n_atoms} p={m.info()['order']} d={m.info()['depth']}: E {e[0]:.2e} F {e[1]:.2e} "
              f"dVdl {e[2]:.2e} tangent {e[3]:.2e}")
        assert max(e[:3]) <= 2e-4 and e[3] <= 4e-4
        m.close()


def test_batch_graph_mode_is_refused():
    """Graph capture is only offered for packed batches; a packed batch refuses
    float64 contexts."""
    import paper_2410_01754_amd as pkg
    systems = make_batch(n_systems=1, n_min=1500, n_max=2000, seed=79)
    mods = _build(systems)
    with pytest.raises(pkg.MahiError) as e:
        pkg.Batch(mods, use_graph=True)
    assert e.value.status == -6
    m64 = _build(systems, precision=64)
    with pytest.raises(pkg.MahiError) as e:
        pkg.Batch(m64, packed=True)
    assert e.value.status == -6
    mods[0].close()
    m64[0].close()
