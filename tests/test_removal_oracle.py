"""Pins of the oracle's particle removal (Sec. 6, Outlook: the identity
operator approximated by a particle's neighbours, its circulation handed to
them, the particle dropped).  Readings: first-order identity moments
(sum g = 1, sum g r = 0, g >= 0; a second moment of non-negative weights
cannot vanish), cost |r/h|^2 + 2^-16 rank^2, candidates closer than r h to
another particle taken greedily in id order with exclusion radius R_full h.

* Lattice with one planted particle: by hand, the site (lower id) goes and
  its circulation splits 1/2 : 1/2 onto its two x-neighbours (cost 1 for
  every opposite pair at distance h; the convex tie-break prefers the pair
  with the middle ranks); I2 grows by exactly Gamma h^2.
* Any cloud: the moment conditions of every removed particle, I0 and I1
  kept, the I2 change equals sum_i Gamma_i sum_j g_ij |x_j - x_i|^2.
* The LP optimum equals brute-force enumeration of all 3-column bases.
* The selection equals a separate greedy pass, and removed particles are
  pairwise farther than R_full h apart.
* Infeasible cases stay: a close pair whose neighbours all lie on one side.
"""
import itertools

import numpy as np
import pytest

import workloads


def _f32d2(xa, ya, xb, yb):
    dx = np.float32(xa) - np.float32(xb)
    dy = np.float32(ya) - np.float32(yb)
    return np.float32(np.float32(dx * dx) + np.float32(dy * dy))


def _inv(x, y, g):
    i0, (i1x, i1y), i2 = _orc_inv(x, y, g)
    return i0, i1x, i1y, i2


def _orc_inv(x, y, g):
    x, y, g = (np.asarray(a, np.float64) for a in (x, y, g))
    return g.sum(), ((g * x).sum(), (g * y).sum()), (g * (x * x + y * y)).sum()


def _bounds(h, rad):
    return np.float32(rad * rad * h * h * (1.0 + 2.0 ** -20)), np.float32(0.25 * h * h * (1.0 - 2.0 ** -20))


def test_lattice_planted_particle_by_hand(orc):
    h = 0.05
    x, y = workloads.lattice(-1.0, 1.0, h)
    n = x.size
    c = int(np.argmin(x * x + y * y))
    x2 = np.append(x, x[c] + 0.3 * h).astype(np.float32).astype(np.float64)
    y2 = np.append(y, y[c]).astype(np.float32).astype(np.float64)
    ids = np.arange(n + 1, dtype=np.int32)
    g = np.full(n + 1, 0.01)
    g[c] = 0.37
    r = orc.remove(x2, y2, g, ids, orc.params(h, q=2))
    assert r.n_candidates == 2
    np.testing.assert_array_equal(r.removed_ids, [c])
    k = r.kcol[c]
    got = {int(r.cols[c, t]): r.g[c, t] for t in range(k) if r.g[c, t] != 0.0}
    assert set(got) == {c - 1, c + 1}
    assert abs(got[c - 1] - 0.5) <= 1e-14 and abs(got[c + 1] - 0.5) <= 1e-14
    i0, i1x, i1y, i2 = _inv(x2, y2, g)
    j0, j1x, j1y, j2 = _inv(r.x, r.y, r.gamma)
    assert abs(j0 - i0) <= 1e-14 and abs(j1x - i1x) <= 1e-14 and abs(j1y - i1y) <= 1e-14
    # I2 grows by Gamma sum_j g_j |x_j - x_c|^2: Gamma h^2 up to the FP32 rounding of the sites
    d = [(x2[j] - x2[c]) ** 2 + (y2[j] - y2[c]) ** 2 for j in (c - 1, c + 1)]
    assert abs((j2 - i2) - 0.37 * 0.5 * (d[0] + d[1])) <= 1e-14
    assert abs(0.5 * (d[0] + d[1]) - h * h) <= 1e-6 * h * h
    # nothing is closer than r h any more: a second pass removes nothing
    r2 = orc.remove(r.x, r.y, r.gamma, r.ids, orc.params(h, q=2))
    assert r2.n_candidates == 0 and r2.removed_ids.size == 0


@pytest.mark.parametrize("q", [2, 3])
def test_moments_and_invariants(orc, q):
    wl = workloads.config_close_pairs(h=0.04, q=q, frac=0.1, seed=7)
    x, y, g = (a.astype(np.float64) for a in (wl.x, wl.y, wl.gamma))
    r = orc.remove(x, y, g, wl.ids, orc.params_of(wl))
    assert r.removed_ids.size > 20
    dI2 = 0.0
    for i in np.flatnonzero(r.kcol):
        k = r.kcol[i]
        cols, f = r.cols[i, :k], r.g[i, :k]
        rx, ry = (x[cols] - x[i]) / wl.h, (y[cols] - y[i]) / wl.h
        assert (f >= 0.0).all() and (f > 0.0).sum() <= 3
        assert abs(f.sum() - 1.0) <= 1e-12
        assert abs(f @ rx) <= 1e-12 and abs(f @ ry) <= 1e-12
        dI2 += g[i] * wl.h ** 2 * (f @ (rx * rx + ry * ry))
    i0, i1x, i1y, i2 = _inv(x, y, g)
    j0, j1x, j1y, j2 = _inv(r.x, r.y, r.gamma)
    s = np.abs(g).sum()
    assert abs(j0 - i0) <= 1e-13 * s
    assert abs(j1x - i1x) <= 1e-13 * s and abs(j1y - i1y) <= 1e-13 * s
    assert abs((j2 - i2) - dI2) <= 1e-13 * s


def _brute(rx, ry, ids):
    """min sum_j c_j g_j over all 3-column bases of [1; rx; ry] g = e0, g >= 0."""
    k = rx.size
    rank = np.array([(ids < ids[t]).sum() for t in range(k)], float)
    c = rx * rx + ry * ry + 2.0 ** -16 * rank * rank
    best, arg = np.inf, None
    for cols in itertools.combinations(range(k), 3):
        B = np.vstack([np.ones(3), rx[list(cols)], ry[list(cols)]])
        if abs(np.linalg.det(B)) < 1e-12:
            continue
        z = np.linalg.solve(B, [1.0, 0.0, 0.0])
        if (z < -1e-12).any():
            continue
        v = c[list(cols)] @ z
        if v < best:
            best, arg = v, (cols, z)
    return best, arg, c


def test_identity_lp_matches_vertex_enumeration(orc):
    wl = workloads.config_close_pairs(h=0.04, q=2, frac=0.1, seed=11)
    x, y, g = (a.astype(np.float64) for a in (wl.x, wl.y, wl.gamma))
    ids = wl.ids
    r = orc.remove(x, y, g, ids, orc.params_of(wl))
    checked = 0
    for i in np.flatnonzero(r.kcol)[:40]:
        k = r.kcol[i]
        cols, f = r.cols[i, :k], r.g[i, :k]
        rx, ry = (x[cols] - x[i]) / wl.h, (y[cols] - y[i]) / wl.h
        best, (bc, bz), c = _brute(rx, ry, ids[cols])
        assert abs(c @ f - best) <= 1e-12 * best
        want = np.zeros(k)
        want[list(bc)] = bz
        np.testing.assert_allclose(f, want, atol=1e-12)
        checked += 1
    assert checked >= 20


def test_selection_is_the_greedy_pass(orc):
    wl = workloads.config_close_pairs(h=0.05, q=2, frac=0.15, seed=5)
    x, y, g = (a.astype(np.float64) for a in (wl.x, wl.y, wl.gamma))
    ids = wl.ids
    P = orc.params_of(wl)
    r = orc.remove(x, y, g, ids, P)
    hi2, lo2 = _bounds(wl.h, wl.R_full)
    n = x.size
    d2 = _f32d2(x[:, None], y[:, None], x[None, :], y[None, :])
    np.fill_diagonal(d2, np.inf)
    cand = np.flatnonzero((d2 < lo2).any(axis=1))
    assert cand.size == r.n_candidates
    taken = []
    for i in cand[np.argsort(ids[cand], kind="stable")]:
        if all(d2[i, j] > hi2 for j in taken):
            taken.append(i)
    removed = set(np.flatnonzero(r.kcol).tolist())
    assert removed <= set(taken)
    # the taken ones that stay have an infeasible identity LP
    for i in set(taken) - removed:
        mem = np.flatnonzero((d2[i] >= lo2) & (d2[i] <= hi2))
        if mem.size >= 3:
            best, _, _ = _brute((x[mem] - x[i]) / wl.h, (y[mem] - y[i]) / wl.h, ids[mem])
            assert not np.isfinite(best)
    for a, b in itertools.combinations(sorted(removed), 2):
        assert d2[a, b] > hi2
    np.testing.assert_array_equal(np.sort(r.removed_ids), np.sort(ids[sorted(removed)]))


def test_one_sided_neighbourhood_stays(orc):
    h = 0.05
    # a row of particles; a close pair at its end has all neighbours on one side
    x = np.concatenate([h * np.arange(10.0), [0.2 * h]])
    y = np.zeros(11)
    ids = np.arange(11, dtype=np.int32)
    g = np.ones(11)
    r = orc.remove(x, y, g, ids, orc.params(h, q=2))
    assert r.n_candidates == 2 and r.removed_ids.size == 0
    np.testing.assert_array_equal(r.gamma, g)
    # an isolated close pair has no neighbourhood at all
    r = orc.remove(np.array([0.0, 0.1 * h]), np.zeros(2), np.ones(2), np.arange(2, dtype=np.int32),
                   orc.params(h, q=2))
    assert r.n_candidates == 2 and r.removed_ids.size == 0


def near_infeasible_cloud(h=0.05, delta=5e-4):
    """A candidate (id 0) whose neighbours (1, -delta) h, (-1, -delta) h, (0, -1) h
    leave the origin delta h outside their hull, and its close partner (id 1)."""
    x = h * np.array([0.0, 0.0, 1.0, -1.0, 0.0])
    y = h * np.array([0.0, 0.3, -delta, -delta, -1.0])
    return x.astype(np.float32).astype(np.float64), y.astype(np.float32).astype(np.float64)


def test_near_infeasible_candidate_stays(orc):
    """Infeasible by delta = 5e-4 h (sum g r_y = 0 needs weight above the line):
    the candidate stays; a phase I stopped within an FP32 tolerance must not
    take it."""
    h = 0.05
    x, y = near_infeasible_cloud(h)
    r = orc.remove(x, y, np.ones(5), np.arange(5, dtype=np.int32), orc.params(h, q=2))
    assert r.n_candidates == 2 and r.removed_ids.size == 0

