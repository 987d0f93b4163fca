"""Pins of the primitive-schedule oracle (Sec. 4.3, Eq. 4-5; supplementary
Eq. 8 and the densification step): the equations' endpoints and steady
state, brute-force top-k, and the split sampling against the covariance
R S S^T R^T of the Gaussian it samples."""
import numpy as np
import pytest

from oracle import densify as D
from oracle import project


def test_eq4_endpoints():
    p0, pf, S = 1000.0, 9000.0, 6000
    assert D.primitive_target(123, S, 1.0, p0, pf) == pytest.approx(pf)       # full resolution
    assert D.primitive_target(0, S, 4.0, p0, pf) == pytest.approx(p0 + (pf - p0) / 16)
    assert D.primitive_target(S, S, 4.0, p0, pf) == pytest.approx(p0 + (pf - p0) / 4)
    # the exponent falls from 2 to 1: at fixed r > 1 the target grows with i
    ts = [D.primitive_target(i, S, 3.0, p0, pf) for i in range(0, S + 1, 500)]
    assert all(b > a for a, b in zip(ts, ts[1:]))


def test_eq5_monotone_and_eq8_steady_state():
    gamma, eta, p_add = 0.98, 1.0, 37.0
    p = 100.0
    seq = []
    for _ in range(2000):
        p = D.budget_update(p, p_add, gamma, eta)
        seq.append(p)
    assert all(b >= a for a, b in zip(seq, seq[1:]))
    assert p == pytest.approx(eta / (1 - gamma) * p_add, rel=1e-9)
    # a budget above the steady state stays where it is (the max keeps it)
    assert D.budget_update(5000.0, p_add, gamma, eta) == 5000.0


def _scene(n, seed):
    rng = np.random.default_rng(seed)
    q = rng.normal(size=(n, 4))
    return dict(means=rng.uniform(-1, 1, (n, 3)), log_scales=rng.normal(-3, 0.7, (n, 3)),
                quats=q, opacity_logits=rng.normal(0, 2, n), sh=rng.normal(0, 0.1, (n, 16, 3)))


def test_top_k_is_brute_force_with_index_ties():
    rng = np.random.default_rng(1)
    score = rng.choice(np.array([0.5, 1.0, 2.0, 3.0], np.float32), 200)
    cand = rng.uniform(size=200) < 0.7
    for k in (0, 1, 17, 90, 500):
        sel = D.select_top(score, cand, k)
        brute = sorted([i for i in range(200) if cand[i]], key=lambda i: (-float(score[i]), i))[:k]
        assert set(np.nonzero(sel)[0]) == set(brute)


def test_densify_counts_layout_and_clones():
    n = 300
    p = _scene(n, 2)
    mom = {f"{t}_{k}": np.random.default_rng(3).normal(size=v.shape) for k, v in p.items()
           for t in ("m", "v")}
    rng = np.random.default_rng(4)
    accum, count = rng.uniform(0, 1, n), rng.integers(0, 4, n).astype(np.float64)
    z = rng.normal(size=(n, 2, 3))
    new, newm, info = D.densify(p, mom, accum, count, z, grad_thr=0.2, min_opacity=0.1,
                                max_scale=0.05, k=40)
    assert info["n_selected"] == 40 and info["n_new"] == n - info["n_pruned"] + 40
    assert info["n_split"] > 0 and info["n_clone"] > 0
    score, prune, cand = D.classify(accum, count, p["opacity_logits"], 0.2, 0.1)
    sel = D.select_top(score, cand, 40)
    o = 0
    for g in range(n):
        if prune[g]:
            continue
        split = sel[g] and np.exp(p["log_scales"][g]).max() > 0.05
        if split:
            assert np.allclose(new["log_scales"][o], p["log_scales"][g] - np.log(1.6))
            assert np.allclose(new["sh"][o + 1], p["sh"][g]) and not newm["m_means"][o].any()
            o += 2
            continue
        assert np.array_equal(new["means"][o], p["means"][g])
        assert np.array_equal(newm["v_quats"][o], mom["v_quats"][g])
        o += 1
        if sel[g]:                                   # clone: an identical copy, fresh moments
            for name in p:
                assert np.array_equal(new[name][o], p[name][g])
            assert not newm["m_sh"][o].any() and not newm["v_opacity_logits"][o].any()
            o += 1
    assert o == info["n_new"]


def test_split_children_sample_the_gaussian():
    """Children at mu + R diag(s) z with z ~ N(0, I) have covariance R S S^T R^T,
    the covariance the projection builds from the same parameters."""
    n = 1
    p = _scene(n, 5)
    p["log_scales"][0] = np.log([0.3, 0.1, 0.05])
    p["opacity_logits"][0] = 3.0
    rng = np.random.default_rng(6)
    pts = []
    for _ in range(6000):
        z = rng.normal(size=(1, 2, 3))
        new, _, _ = D.densify(p, {}, np.ones(1), np.ones(1), z, 0.5, 0.01, 0.01, 1)
        pts.append(new["means"])
    pts = np.concatenate(pts) - p["means"][0]
    q = p["quats"][0] / np.linalg.norm(p["quats"][0])
    M = project.quat_to_rot(q[None])[0] @ np.diag(np.exp(p["log_scales"][0]))
    assert np.abs(np.cov(pts.T) - M @ M.T).max() < 0.05 * np.abs(M @ M.T).max()
    assert np.abs(pts.mean(axis=0)).max() < 0.02
