"""Pins of the oracle's non-negative least-squares stencils (the alternative to
the simplex that Sec. 4.1 discusses: min_{f >= 0} |V f - b|^2, Lawson-Hanson).

* The optimality (KKT) conditions of NNLS on random problems: f >= 0, the
  negative gradient w = V^T (b - V f) vanishes on the support and is <= 0 off it.
* The optimum against an independent solver (scipy.optimize.nnls) and, on tiny
  problems, against brute force over every support (the unconstrained least
  squares on each column subset, kept when non-negative): the same residual.
* On moment problems (Sec. 2 eqs. cond_two/cond_alpha) that have a non-negative
  solution the residual vanishes, so the stencil meets the moment conditions;
  it has at most m non-zero fractions, and the lemma of Sec. 3.2 holds.
* A whole run with NNLS stencils keeps I0 exactly and approximates the
  Lamb-Oseen solution as well as the canonical stencils.
"""
import itertools

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _moment_matrix(rx, ry, q):
    rows = [rx, ry, rx * rx, rx * ry, ry * ry]
    if q == 3:
        rows += [rx ** 3, rx * rx * ry, rx * ry * ry, ry ** 3]
    return np.array(rows)


def _kkt(A, b, f, tol):
    w = A.T @ (b - A @ f)
    on = f > 0
    return (f >= 0).all() and (np.abs(w[on]) <= tol).all() and (w[~on] <= tol).all()


@pytest.mark.parametrize("seed", range(6))
def test_nnls_kkt_and_scipy(orc, seed):
    from scipy.optimize import nnls as scipy_nnls
    rng = np.random.default_rng(seed)
    for trial in range(40):
        m = int(rng.choice([3, 5, 9]))
        k = int(rng.integers(m, 30))
        A = rng.normal(size=(m, k))
        b = rng.normal(size=m) if trial % 2 else A @ (np.abs(rng.normal(size=k)) * (rng.random(k) < 0.4))
        f, adds = orc.nnls(A, b)
        tol = 1e-9 * np.abs(A).max() * max(1.0, np.abs(b).max()) * m
        assert _kkt(A, b, f, tol), (seed, trial)
        fs, rs = scipy_nnls(A, b)
        assert np.linalg.norm(A @ f - b) <= rs + 1e-9 * (1 + np.abs(b).max())


def test_nnls_brute_force_over_supports(orc):
    rng = np.random.default_rng(11)
    for trial in range(60):
        m = int(rng.choice([3, 5]))
        k = int(rng.integers(m, 9))
        A = rng.normal(size=(m, k))
        b = rng.normal(size=m)
        f, _ = orc.nnls(A, b)
        best = np.linalg.norm(b)
        for p in range(1, m + 1):
            for S in itertools.combinations(range(k), p):
                z, *_ = np.linalg.lstsq(A[:, S], b, rcond=None)
                if (z >= 0).all():
                    best = min(best, np.linalg.norm(A[:, S] @ z - b))
        assert abs(np.linalg.norm(A @ f - b) - best) <= 1e-9 * (1 + best), trial


@pytest.mark.parametrize("q", [2, 3])
def test_nnls_moment_stencils(orc, q):
    """Moment problems of a jittered cloud with a non-negative solution: NNLS returns
    a stencil (zero residual), non-negative, with at most m non-zeros, and the
    Sec. 3.2 lemma holds (sum f |r|^2 = 4, 4 / R^2 <= sum f <= 4 / r^2)."""
    wl = workloads.config_jittered(h=0.05, q=q, seed=3)
    mask, _, _ = orc.diffused(wl.gamma, wl.ids, wl.h, wl.q)
    P = orc.params_of(wl, solver=1)
    st = orc.stencils(wl.x, wl.y, wl.ids, mask, P)
    ref = orc.stencils(wl.x, wl.y, wl.ids, mask, orc.params_of(wl))
    m = 5 if q == 2 else 9
    ok = np.flatnonzero(st.status <= 1)
    assert ok.size > 100
    # NNLS finds a stencil wherever the LP does (both decide feasibility of the same system)
    np.testing.assert_array_equal(st.status <= 1, ref.status <= 1)
    x, y = wl.x.astype(np.float64), wl.y.astype(np.float64)
    for i in ok:
        cols, f = st.cols[i, :st.kcol[i]], st.f[i, :st.kcol[i]]
        rx, ry = (x[cols] - x[i]) / wl.h, (y[cols] - y[i]) / wl.h
        A = _moment_matrix(rx, ry, q)
        b = np.zeros(m)
        b[2] = b[4] = 2.0
        assert np.abs(A @ f - b).max() <= 1e-10
        assert (f >= 0).all() and (f > 0).sum() <= m
        r2 = rx * rx + ry * ry
        assert abs((f * r2).sum() - 4.0) <= 1e-9
        R = wl.R_full if st.status[i] == 1 else wl.R
        assert 4.0 / (R * R) - 1e-9 <= f.sum() <= 16.0 + 1e-9
        assert abs(st.fii[i] + f.sum()) <= 1e-12


def test_nnls_run_conserves_and_converges(orc):
    """Whole runs with NNLS stencils: I0 kept to 1e-12, and the weak error against the
    Lamb-Oseen closed form within a factor 1.5 of the canonical stencils' (Sec. 5)."""
    from test_oracle_pins import _weak_error
    wl = workloads.config_jittered(h=0.04, q=2, seed=2)
    steps = 10
    out = []
    for solver in (0, 1):
        st = orc.initial_state(wl)
        P = orc.params_of(wl, solver=solver)
        for _ in range(steps):
            st = orc.step(st, wl, params=P)
        assert abs(st.gamma.sum() - wl.gamma.astype(np.float64).sum()) <= 1e-12
        out.append(_weak_error(st.x, st.y, st.gamma, wl.t0 + steps * wl.dt, wl.nu))
    assert out[1] <= 1.5 * out[0], out
