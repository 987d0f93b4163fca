"""The densification step on the device against the oracle (Sec. 4.3;
supplementary "Densification of DashGaussian"): counts, the selected top k
with index tie-break, the output layout, copies, split children and moments.
Seeded inputs; opacities and scales are kept off the float32 decision
thresholds so both sides take every integer decision alike."""
import numpy as np
import pytest
import torch

from oracle import densify as OD
from paper_2503_18402_amd import densify, gsmi, raster

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    p = dict(means=rng.uniform(-1, 1, (n, 3)), log_scales=rng.normal(-3, 0.7, (n, 3)),
             quats=rng.normal(size=(n, 4)), opacity_logits=rng.normal(0, 2.5, n),
             sh=rng.normal(0, 0.1, (n, 16, 3)))
    p = {k: v.astype(np.float32) for k, v in p.items()}
    # keep decisions away from the thresholds (sigmoid 0.05, scale 0.08)
    logit_min = np.float32(np.log(0.05 / 0.95))
    near = np.abs(p["opacity_logits"] - logit_min) < 1e-3
    p["opacity_logits"][near] += np.float32(0.01)
    ls_max = np.float32(np.log(0.08))
    near = np.abs(p["log_scales"] - ls_max) < 1e-3
    p["log_scales"][near] -= np.float32(0.01)
    mom = {f"{t}_{k}": rng.normal(size=v.shape).astype(np.float32) for k, v in p.items()
           for t in ("m", "v")}
    accum = rng.uniform(0, 2, n).astype(np.float32)
    count = rng.integers(0, 5, n).astype(np.float32)
    accum[: n // 10] = np.float32(3.0)          # 2000 ties at score 1.5: the cutoff of
    count[: n // 10] = np.float32(2.0)          # k = 1500 falls inside them
    z = rng.normal(size=(n, 2, 3)).astype(np.float32)
    return p, mom, accum, count, z


@pytest.mark.parametrize("k", [0, 500, 1500, 10 ** 9])
def test_densify_step_matches_oracle(k):
    n = 20000
    p, mom, accum, count, z = _inputs(n, 81 + (k % 7))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    P = {name: dev(v) for name, v in p.items()}
    M = {name: dev(mom["m_" + name]) for name in raster.PARAM_NAMES}
    V = {name: dev(mom["v_" + name]) for name in raster.PARAM_NAMES}
    newp, newm, newv, info = densify.densify_step(P, M, V, dev(accum), dev(count), dev(z),
                                                  0.3, 0.05, 0.08, lambda kept, cand: k)
    torch.cuda.synchronize()
    ref, refm, rinfo = OD.densify({k_: v.astype(np.float64) for k_, v in p.items()},
                                  {k_: v.astype(np.float64) for k_, v in mom.items()},
                                  accum, count, z.astype(np.float64), 0.3, 0.05, 0.08, k)
    assert info["n_pruned"] == rinfo["n_pruned"] and info["n_candidates"] == rinfo["p_add"]
    assert info["n_new"] == rinfo["n_new"]
    if k == 500:
        assert 0 < rinfo["n_split"] and 0 < rinfo["n_clone"]
    for name in raster.PARAM_NAMES:
        got = newp[name].cpu().numpy().astype(np.float64)
        assert got.shape == ref[name].shape, name
        tol = 1e-5 if name in ("means", "log_scales") else 0.0
        assert np.abs(got - ref[name]).max() <= tol * max(1.0, np.abs(ref[name]).max()), name
        assert np.array_equal(newm[name].cpu().numpy(), refm["m_" + name].astype(np.float32))
        assert np.array_equal(newv[name].cpu().numpy(), refm["v_" + name].astype(np.float32))


def test_stats_accumulate_seen_views():
    """accum += |d mean2D|, count += views with a footprint, untouched otherwise."""
    from paper_2503_18402_amd import scenes
    sc = scenes.make_scene(3000, seed=85, mean_range=1.0)
    sc["means"][:50] = (0.0, 50.0, 0.0)  # outside every view
    base = scenes.orbit_cameras(3, 3.0, 96, 64, 90.0)
    params = raster.to_device(sc, "cuda")
    frame = raster.render(params, base)
    n = params["means"].shape[0]
    mabs = torch.rand(n, device="cuda")
    accum = torch.full((n,), 0.5, device="cuda")
    count = torch.ones(n, device="cuda")
    gsmi.gs_densify_stats(3, n, frame.proj, mabs, accum, count)
    torch.cuda.synchronize()
    tt = frame.proj.cpu().numpy()
    from tests import gpu_util as U
    seen = sum((U.decode_proj(frame, view=v)["tt"] > 0).astype(np.float32) for v in range(3))
    exp_c = 1.0 + seen
    exp_a = 0.5 + np.where(seen > 0, mabs.cpu().numpy(), 0.0)
    assert np.array_equal(count.cpu().numpy(), exp_c.astype(np.float32))
    assert np.array_equal(accum.cpu().numpy(), exp_a.astype(np.float32))
    assert (seen[:50] == 0).all() and (seen[50:] > 0).any()
