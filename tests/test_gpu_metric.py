"""GPU parity of the accuracy metric (Sec. III-D, mrf_accuracy) against the FP64
oracle on the same map.  The map comes from the oracle's inference (or a seeded
generator), rounded to float32, and both sides take every decision in FP64:
ray codes and chosen surface depths agree exactly wherever the oracle's
decision is more than 1e-9 (in log omega, or log visibility against the
threshold) from a tie; evaluated-ray counts agree exactly."""
import math

import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NEAR_TIE = 1e-9


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def RayMRF():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2006_03512_amd.mrf import RayMRF as R
    return R


def _scene(name):
    if name.startswith("rand"):
        return S.random_scene(int(name[4:]))
    return S.make(name)


def _expected_surface(a):
    return np.where(np.isinf(a["t_out"]), np.inf, a["t_in"])


def _compare(a, code, surf):
    """Oracle result a (one scene) against the GPU's code / surface arrays."""
    ev = a["code"] >= 0
    np.testing.assert_array_equal(code >= 0, ev)                      # which rays are evaluated
    assert np.all(np.isnan(surf[~ev]))
    clear = ev & (a["margin"] > NEAR_TIE)
    np.testing.assert_array_equal(code[clear], a["code"][clear])
    np.testing.assert_array_equal(surf[clear], _expected_surface(a)[clear])
    ties = int((ev & ~clear).sum())
    assert int((code[ev] != a["code"][ev]).sum()) <= ties
    return int(ev.sum()), int((a["code"] == 1).sum()), ties


@pytest.mark.parametrize("name,sweeps", [("c1", 5), ("fd", 8), ("rand1", 5), ("c2", 10)])
def test_accuracy_of_the_inferred_map(oracle, RayMRF, name, sweeps):
    _say(f"[accuracy] {name} K={sweeps}")
    sc = _scene(name)
    G = oracle.build_graph(sc)
    ref = oracle.infer(G, sc.prior_logit().astype(np.float64), sc.sigma_table, sweeps)
    L32 = ref.L.astype(np.float32)
    a = oracle.accuracy(sc, L32.astype(np.float64))
    m = RayMRF()
    m.build(sc, keep_chords=False)
    out = m.accuracy(torch.from_numpy(L32).cuda())
    code = out["code"].cpu().numpy()
    surf = out["surface_depth"].cpu().numpy()
    n_ev, n_ok, ties = _compare(a, code, surf)
    cnt = out["counts"].cpu().numpy()
    assert cnt[0, 0] == n_ev and cnt[0, 1] == int((code == 1).sum())
    assert abs(int(cnt[0, 1]) - n_ok) <= ties
    assert n_ev > 0
    _say(f"  evaluated {n_ev}, accurate {cnt[0, 1]} ({out['accuracy'][0]:.3f}), near ties {ties}")


def test_accuracy_multi_scene_batch(oracle, RayMRF):
    """Scenes of a batch are evaluated against their own voxels; ray ids and
    counts per scene."""
    scs = [S.make_c1(), S.make_fd(), S.random_scene(4)]
    for s in scs[1:]:
        s.params = scs[0].params
    rng = np.random.default_rng(60)
    Ls = [rng.uniform(-4.0, 4.0, s.grid.n_voxels).astype(np.float32) for s in scs]
    m = RayMRF()
    m.build(scs, keep_chords=False)
    out = m.accuracy(torch.from_numpy(np.concatenate(Ls)).cuda(), vis_min=0.3)
    code = out["code"].cpu().numpy()
    surf = out["surface_depth"].cpu().numpy()
    cnt = out["counts"].cpu().numpy()
    r0 = 0
    for i, (s, L) in enumerate(zip(scs, Ls)):
        a = oracle.accuracy(s, L.astype(np.float64), vis_min=0.3)
        R = s.n_rays
        n_ev, n_ok, ties = _compare(a, code[r0:r0 + R], surf[r0:r0 + R])
        assert cnt[i, 0] == n_ev and abs(int(cnt[i, 1]) - n_ok) <= ties
        r0 += R
    assert r0 == code.shape[0]


def test_accuracy_column_cases(RayMRF):
    """Hand-derived single-column cases (a region of p = 0.7 hides a voxel of
    p = 0.95 behind it; p = 0.2 does not; an empty map leaves the ray visible)."""
    def column(Z):
        T = np.eye(4)
        T[:3, 3] = (0.05, 0.05, -0.5)
        p = S.BuildParams(z_min=0.1, z_max=10.0, trunc_nsigma=3.0, trunc_c0=0.01, trunc_c2=0.0,
                          trunc_min=0.0, table_dmax=8.0, min_ray_voxels=2)
        return S.Scene("column", np.full((1, 1, 1), Z, np.float32), T[None], S.Intrinsics(1, 1, 1.0, 1.0, 0.0, 0.0),
                       S.Grid(1, 1, 16, 0.1), np.zeros((0, 2, 3)), p, np.full(64, 0.01))

    lg = lambda p: math.log(p / (1.0 - p))
    front = np.full(16, -30.0, np.float32)
    front[3:6] = lg(0.7)
    front[8] = lg(0.95)
    thin = np.full(16, -30.0, np.float32)
    thin[3:6] = lg(0.2)
    thin[8] = lg(0.95)
    empty = np.full(16, -30.0, np.float32)
    cases = [(front, 0.85, 1, 0.8), (front, 1.35, 0, 0.8), (thin, 1.35, 1, 1.3), (thin, 0.85, 0, 1.3),
             (empty, 2.5, 1, math.inf), (empty, 1.0, 0, math.inf)]
    zero = np.full(16, -1000.0, np.float32)        # alpha = 0 exactly: exit visibility 1
    cases += [(zero, 2.5, 1, math.inf, 1.0), (zero, 1.0, 0, math.inf, 1.0)]
    m = RayMRF()
    for case in cases:
        L, Z, want, depth = case[:4]
        vis_min = case[4] if len(case) > 4 else 0.5
        m.build(column(Z), keep_chords=False)
        out = m.accuracy(torch.from_numpy(L).cuda(), vis_min=vis_min)
        assert int(out["code"][0]) == want, (Z, want)
        assert float(out["surface_depth"][0]) == pytest.approx(depth, abs=1e-12)
        assert out["counts"].cpu().numpy().tolist() == [[1, want]]


def test_accuracy_of_last_marginals_and_errors(RayMRF):
    from paper_2006_03512_amd import _lib
    sc = S.make_fd()
    m = RayMRF()
    m.build(sc, keep_chords=False)
    with pytest.raises(_lib.MRFError) as ei:
        m.accuracy()                         # no map and no inference yet
    assert ei.value.code == _lib.MRF_ESTATE
    th = torch.from_numpy(sc.prior_logit()).cuda()
    m.infer(th, torch.from_numpy(sc.sigma_table.astype(np.float32)).cuda(), 6)
    _, logit = m.marginals()
    a = m.accuracy()
    b = m.accuracy(logit)
    assert torch.equal(a["code"], b["code"]) and torch.equal(a["counts"], b["counts"])
    for bad in (0.0, -0.1, 1.5, float("nan")):
        with pytest.raises(_lib.MRFError) as ei:
            m.accuracy(logit, vis_min=bad)
        assert ei.value.code == _lib.MRF_EINVAL
