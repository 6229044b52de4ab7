"""Pins of the adaptive-density-control oracle (oracle/adc.py) against hand
cases, invariants and the sampling law; CPU only."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

from oracle import adc

TH = dict(grad_threshold=0.5, split_scale=0.05, prune_density=0.01, prune_scale=0.3)


def _scene():
    # 0: keep (low score); 1: prune (density); 2: clone (score 1.0, small);
    # 3: split (score 2.0, large); 4: prune (too large); 5: keep (never seen)
    ls = np.log(np.array([[0.02, 0.02, 0.01, 0.10, 0.40, 0.02],
                          [0.02, 0.02, 0.01, 0.04, 0.01, 0.02],
                          [0.02, 0.02, 0.01, 0.04, 0.01, 0.02]]))
    gs = dict(mean=np.arange(18, dtype=np.float64).reshape(3, 6) / 10.0, log_scale=ls,
              quat=np.tile(np.array([[1.0], [0.0], [0.0], [0.0]]), (1, 6)),
              density=np.array([0.3, 0.001, 0.4, 0.8, 0.5, 0.2]))
    stat = np.array([[0.2, 5.0, 3.0, 4.0, 9.0, 0.0],
                     [1.0, 1.0, 3.0, 2.0, 1.0, 0.0]])
    m = {k: v + 100.0 for k, v in gs.items()}
    v = {k: v + 200.0 for k, v in gs.items()}
    return gs, stat, m, v


def test_hand_case_decisions_order_and_values():
    gs, stat, m, v = _scene()
    z = np.zeros((6, 6))
    z[0, 3] = 1.0    # first child +1 sigma along x
    z[3, 3] = -1.0   # second child -1 sigma along x
    out, mo, vo, code = adc.densify(gs, m, v, stat, z, **TH, split_shrink=2.0, n_max=10)
    assert code.tolist() == [adc.KEEP, adc.PRUNE, adc.CLONE, adc.SPLIT, adc.PRUNE, adc.KEEP]
    # survivors 0, 2, 2', 3a, 3b, 5
    assert out["density"].tolist() == [0.3, 0.2, 0.2, 0.8 * 8 / 2, 0.8 * 8 / 2, 0.2]
    np.testing.assert_allclose(out["mean"][:, 3], gs["mean"][:, 3] + [0.10, 0, 0], atol=1e-15)
    np.testing.assert_allclose(out["mean"][:, 4], gs["mean"][:, 3] - [0.10, 0, 0], atol=1e-15)
    np.testing.assert_allclose(np.exp(out["log_scale"][:, 3]), [0.05, 0.02, 0.02])
    np.testing.assert_allclose(out["mean"][:, [0, 1, 2, 5]], gs["mean"][:, [0, 2, 2, 5]])
    # moments: every output Gaussian carries its source's
    assert mo["density"].tolist() == [100.3, 100.4, 100.4, 100.8, 100.8, 100.2]
    assert vo["density"].tolist() == [200.3, 200.4, 200.4, 200.8, 200.8, 200.2]


def test_cap_keeps_the_largest_scores_ties_by_index():
    gs, stat, m, v = _scene()
    # survivors 0, 2, 3, 5 (4 of them); room for one densification at n_max = 5
    out, _, _, code = adc.densify(gs, m, v, stat, np.zeros((6, 6)), **TH, n_max=5)
    assert code.tolist() == [adc.KEEP, adc.PRUNE, adc.KEEP, adc.SPLIT, adc.PRUNE, adc.KEEP]
    assert out["density"].shape == (5,)
    # equal scores: the lower index wins
    stat2 = stat.copy()
    stat2[:, 3] = [3.0, 3.0]
    _, _, _, code = adc.densify(gs, m, v, stat2, np.zeros((6, 6)), **TH, n_max=5)
    assert code[2] == adc.CLONE and code[3] == adc.KEEP
    # no room at all: nothing is densified; below the survivors: refused
    _, _, _, code = adc.densify(gs, m, v, stat, np.zeros((6, 6)), **TH, n_max=4)
    assert adc.CLONE not in code and adc.SPLIT not in code
    try:
        adc.densify(gs, m, v, stat, np.zeros((6, 6)), **TH, n_max=3)
        raise AssertionError("expected a refusal")
    except ValueError:
        pass


def test_mass_is_preserved_by_clone_and_split():
    rng = np.random.default_rng(3)
    n = 400
    gs = dict(mean=rng.uniform(-0.3, 0.3, (3, n)), log_scale=np.log(rng.uniform(0.005, 0.1, (3, n))),
              quat=rng.normal(size=(4, n)), density=rng.uniform(0.05, 1.0, n))
    stat = np.stack([rng.uniform(0, 2, n), np.ones(n)])
    zeros = {k: np.zeros_like(v) for k, v in gs.items()}
    out, _, _, code = adc.densify(gs, zeros, zeros, stat, rng.normal(size=(6, n)), **TH, n_max=2 * n)
    assert np.sum(code == adc.SPLIT) > 20 and np.sum(code == adc.CLONE) > 20
    kept = {k: v[..., code != adc.PRUNE] for k, v in gs.items()}
    assert math.isclose(adc.mass(out), adc.mass(kept), rel_tol=1e-12)


def test_split_children_follow_the_parent_distribution():
    """Children of one parent, drawn with many normal pairs, have the
    parent's mean and covariance R diag(s^2) R^T."""
    rng = np.random.default_rng(4)
    n = 20000
    q = rng.normal(size=4)
    s = np.array([0.08, 0.03, 0.06])
    gs = dict(mean=np.tile([[0.1], [-0.2], [0.05]], (1, n)), log_scale=np.tile(np.log(s)[:, None], (1, n)),
              quat=np.tile(q[:, None], (1, n)), density=np.full(n, 0.5))
    stat = np.stack([np.ones(n), np.ones(n)])
    zeros = {k: np.zeros_like(v) for k, v in gs.items()}
    out, _, _, code = adc.densify(gs, zeros, zeros, stat, rng.normal(size=(6, n)), **TH, n_max=2 * n)
    assert np.all(code == adc.SPLIT)
    x = out["mean"] - gs["mean"][:, :1]
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    cov = R @ np.diag(s ** 2) @ R.T
    np.testing.assert_allclose(x.mean(axis=1), 0.0, atol=4 * 0.08 / math.sqrt(2 * n))
    np.testing.assert_allclose(np.cov(x), cov, atol=4 * 0.08 ** 2 * math.sqrt(2.0 / (2 * n)))


def test_rotation_matches_scipy_and_accumulate_by_hand():
    q = np.random.default_rng(5).normal(size=(4, 7))
    R = adc.rotation(q)
    for i in range(7):
        ref = Rotation.from_quat([q[1, i], q[2, i], q[3, i], q[0, i]]).as_matrix()
        np.testing.assert_allclose(R[:, :, i], ref, atol=1e-14)
    g = np.array([[3.0, 0.0], [4.0, 0.0], [0.0, 0.0]])
    st = adc.accumulate(g, np.array([[1.0, 2.0], [1.0, 0.0]]))
    assert st.tolist() == [[6.0, 2.0], [2.0, 0.0]]
