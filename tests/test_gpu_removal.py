"""Particle removal (Sec. 6, outlook; `vrm_remove_particles`) on the GPU,
through the C ABI, against the FP64 oracle on the same FP32 inputs.

* Integer work bit-exact: the candidate count, which particles are removed,
  which stay (ids), and the kept positions.
* Circulation within 1e-5 relative L2 (the received g_j Gamma_i are added in
  FP32); I0 and I1 kept to FP32 round-off.
* Both orders of the cloud: as given (the cell list permutes it) and already
  in cell order (after a step).
* Edges: empty cloud, one particle, no candidates, an isolated close pair,
  repeated calls until nothing is close, and a step after a removal.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vrm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1508_06379_amd as v
    v.lib()
    return v


def _say(*a):
    print(*a, flush=True)


def _planted_lattice():
    h = 0.05
    x, y = workloads.lattice(-1.0, 1.0, h)
    c = int(np.argmin(x * x + y * y))
    x = np.append(x, x[c] + 0.3 * h).astype(np.float32)
    y = np.append(y, y[c]).astype(np.float32)
    wl = workloads.config_lattice_small()
    g = np.append(wl.gamma, np.float32(0.01))
    return workloads.Workload("planted_lattice", x, y, g.astype(np.float32), h=h, nu=wl.nu, q=2, dt=wl.dt,
                              steps=0, t0=wl.t0)


CASES = {
    "planted_lattice": _planted_lattice,
    "close_pairs_h0.04_q2": lambda: workloads.config_close_pairs(h=0.04, q=2, frac=0.1, seed=7),
    "close_pairs_h0.02_q2": lambda: workloads.config_close_pairs(h=0.02, q=2),
    "close_pairs_h0.02_q3": lambda: workloads.config_close_pairs(h=0.02, q=3, frac=0.08, seed=9),
    "close_pairs_h0.01_q2": lambda: workloads.config_close_pairs(h=0.01, q=2),
}


def _gpu_remove(vrm, wl, after_step=False):
    P = vrm.params_of(wl)
    cloud = vrm.Cloud(wl.x, wl.y, wl.gamma, capacity=3 * wl.n + 64)
    ctx = vrm.Context(cloud.capacity)
    if after_step:
        # puts the cloud in cell order with a valid cell list (zero dt: nothing moves)
        Pz = vrm.params_of(wl)
        Pz.dt = 0.0
        ctx.vrm_insert_particles(cloud, Pz)
    x0, y0, g0, i0 = cloud.numpy()
    nr, nc = ctx.vrm_remove_particles(cloud, P)
    torch.cuda.synchronize()
    return (x0, y0, g0, i0), cloud.numpy(), nr, nc, (ctx, cloud, P)


def _compare(orc, wl, before, after, nr, nc):
    x0, y0, g0, i0 = before
    ref = orc.remove(x0.astype(np.float64), y0.astype(np.float64), g0.astype(np.float64), i0, orc.params_of(wl))
    x, y, g, ids = after
    _say(wl.name, "N", x0.size, "candidates", nc, ref.n_candidates, "removed", nr, ref.removed_ids.size)
    assert nc == ref.n_candidates
    assert nr == ref.removed_ids.size
    assert x.size == x0.size - nr
    o, ro = np.argsort(ids), np.argsort(ref.ids)
    np.testing.assert_array_equal(ids[o], ref.ids[ro])
    np.testing.assert_array_equal(x[o], ref.x[ro].astype(np.float32))
    np.testing.assert_array_equal(y[o], ref.y[ro].astype(np.float32))
    err = np.linalg.norm(g[o].astype(np.float64) - ref.gamma[ro]) / np.linalg.norm(ref.gamma)
    s = np.abs(g0.astype(np.float64)).sum()
    d0 = abs(g.astype(np.float64).sum() - g0.astype(np.float64).sum())
    d1 = abs((g.astype(np.float64) * x).sum() - (g0.astype(np.float64) * x0).sum())
    _say("  rel L2", err, "dI0", d0, "dI1x", d1)
    assert err <= 1e-5
    assert d0 <= 1e-6 * s and d1 <= 1e-6 * s


@pytest.mark.parametrize("name", list(CASES))
def test_removal_matches_oracle(vrm, orc, name):
    wl = CASES[name]()
    _say("case", name, wl.n)
    before, after, nr, nc, _ = _gpu_remove(vrm, wl)
    assert nr > 0
    _compare(orc, wl, before, after, nr, nc)


def test_removal_on_a_cloud_in_cell_order(vrm, orc):
    wl = workloads.config_close_pairs(h=0.02, q=2, seed=12)
    before, after, nr, nc, _ = _gpu_remove(vrm, wl, after_step=True)
    assert nr > 0
    _compare(orc, wl, before, after, nr, nc)


def test_removal_at_larger_size(vrm, orc):
    """680 k particles over [-2, 2]^2 at h = 0.005 (the oracle does all of them)."""
    wl = workloads.config_close_pairs(h=0.005, q=2, lo=-2.0, hi=2.0, seed=21)
    _say("case close_pairs_h0.005", wl.n)
    before, after, nr, nc, _ = _gpu_remove(vrm, wl)
    _compare(orc, wl, before, after, nr, nc)


def test_repeated_removal_until_nothing_is_close_then_step(vrm, orc):
    wl = workloads.config_close_pairs(h=0.02, q=2, frac=0.2, seed=3)
    before, after, nr, nc, (ctx, cloud, P) = _gpu_remove(vrm, wl)
    total, calls = nr, 1
    while nc > 0 and calls < 20:
        st = cloud.numpy()
        nr, nc = ctx.vrm_remove_particles(cloud, P)
        _compare(orc, wl, st, cloud.numpy(), nr, nc)
        total += nr
        calls += 1
        if nr == 0:
            break
    _say("calls", calls, "removed", total, "left candidates", nc)
    assert total > 0
    # the context's cached state follows the compaction: a step still conserves I0,
    # and the particles it inserts get ids above every surviving one (Sec. 4.2 as
    # the oracle does it: max id + 1, ...), so all ids stay distinct
    x, y, g, ids = cloud.numpy()
    s0 = g.astype(np.float64).sum()
    mask, _, _ = orc.diffused(g.astype(np.float64), ids, wl.h, wl.q, wl.c_diff)
    rx, ry, rg, rids, _ = orc.insert(x.astype(np.float64), y.astype(np.float64), g.astype(np.float64), ids, mask,
                                     orc.params_of(wl))
    ctx.vrm_step(cloud, P, None, wl.t0)
    torch.cuda.synchronize()
    x2, y2, g2, ids2 = cloud.numpy()
    assert abs(g2.astype(np.float64).sum() - s0) <= 1e-5 * np.abs(g).sum()
    _say("after the removals: N", x.size, "max id", ids.max(), "inserted by the step", x2.size - x.size,
         "oracle", rx.size - x.size)
    assert x2.size > x.size and x.size > 0
    assert np.unique(ids2).size == ids2.size
    o, ro = np.argsort(ids2), np.argsort(rids)
    np.testing.assert_array_equal(ids2[o], rids[ro])
    # the new particles sit where the oracle put them (the stage moves nothing: u = 0)
    np.testing.assert_array_equal(x2[o], rx[ro].astype(np.float32))
    np.testing.assert_array_equal(y2[o], ry[ro].astype(np.float32))


def test_removal_edges(vrm, orc):
    h = 0.05
    wl = workloads.config_lattice_small()
    P = vrm.params_of(wl)
    # no candidates: the cloud is unchanged
    cloud = vrm.Cloud(wl.x, wl.y, wl.gamma, capacity=wl.n + 64)
    ctx = vrm.Context(cloud.capacity)
    before = cloud.numpy()
    assert ctx.vrm_remove_particles(cloud, P) == (0, 0)
    after = cloud.numpy()
    for a, b in zip(before, after):
        np.testing.assert_array_equal(a, b)
    # empty, one particle, an isolated close pair (no neighbourhood: stays)
    for xs in ([], [0.0], [0.0, 0.1 * h]):
        x = np.array(xs, np.float32)
        cl = vrm.Cloud(x, np.zeros_like(x), np.ones_like(x), capacity=16)
        cx = vrm.Context(16)
        nr, nc = cx.vrm_remove_particles(cl, P)
        assert nr == 0 and nc == (2 if len(xs) == 2 else 0) and cl.n == len(xs)
    with pytest.raises(vrm.VrmError):
        bad = vrm.params_of(wl)
        bad.h = -1.0
        ctx.vrm_remove_particles(cloud, bad)


def test_near_infeasible_candidate_stays(vrm, orc):
    """Regression: phase I ends within its FP32 tolerance (5e-4 of the rhs) on a
    vertex with a non-zero artificial; certification must reject it."""
    from test_removal_oracle import near_infeasible_cloud
    h = 0.05
    x, y = near_infeasible_cloud(h)
    wl = workloads.Workload("near_infeasible", x.astype(np.float32), y.astype(np.float32),
                            np.ones(5, np.float32), h=h, nu=0.01, q=2, dt=0.0, steps=0)
    before, after, nr, nc, _ = _gpu_remove(vrm, wl)
    assert nc == 2 and nr == 0
    _compare(orc, wl, before, after, nr, nc)

