"""GPU: every candidate launch shape of every ray-length class (the schedule
the autotuner chooses from) gives the oracle's marginals and gradients, and the
autotuner keeps parity.  Scenes with flat, wide grids give tiles of up to ~540
steps, so the classes up to 640 steps all have work; the room frame covers the
short classes."""
import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_P = 1e-4
TOL_G = 1e-3
TILE_CLASS_CAPS = [16, 64, 128, 192, 256, 320, 384, 512, 640, 768, 1024, 1536, 2048]


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def RayMRF():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2006_03512_amd.mrf import RayMRF as R
    return R


def _long_ray_scenes():
    """Also used by the CPU test that checks which tile classes they reach."""
    return [S.random_scene(21, grid=(400, 400, 24), voxel=0.01, n_frames=2),
            S.random_scene(22, grid=(320, 320, 40), voxel=0.0125, n_frames=2),
            S.random_scene(23, grid=(480, 480, 20), voxel=0.01, n_frames=2)]


def _grad_rel(g, ref):
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    if not np.any(ref):
        return float(np.abs(g).max())
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    ent = np.abs(g - ref) / (np.abs(ref) + np.abs(ref).max())
    return max(rel, ent.max())


def _reference(oracle, sc, K):
    G = oracle.build_graph(sc)
    th = sc.prior_logit()
    y = sc.occupancy()
    ref = oracle.infer(G, th.astype(np.float64), sc.sigma_table, K, keep_history=True)
    tb, sb, _ = oracle.backward(G, ref, oracle.bce_logit_grad(ref.L, y), sc.sigma_table)
    return ref, tb, sb


def _gpu_run(m, sc, K):
    th = torch.from_numpy(sc.prior_logit()).cuda()
    sig = torch.from_numpy(sc.sigma_table.astype(np.float32)).cuda()
    m.infer(th, sig, K, keep_checkpoints=True)
    p, logit = m.marginals()
    y = torch.from_numpy(sc.occupancy()).cuda()
    gl = (torch.sigmoid(logit) - y) / p.numel()   # d mean-BCE / d logit
    dth, dsg = m.backward(gl.contiguous())
    torch.cuda.synchronize()
    return p.cpu().numpy(), dth.cpu().numpy(), dsg.cpu().numpy()


def test_every_shape_matches_oracle(oracle, RayMRF):
    scs = _long_ray_scenes() + [S.make_c1()]
    K = 4
    for sc in scs:
        ref, tb_ref, sb_ref = _reference(oracle, sc, K)
        m = RayMRF()
        m.build(sc)
        t = m.tuning()
        assert t["cap"] == TILE_CLASS_CAPS
        n_f, n_a = t["fwd_candidates"], t["adj_candidates"]
        for i in range(max(max(n_f), max(n_a))):
            fs = [min(i, n - 1) for n in n_f]
            as_ = [min(i, n - 1) for n in n_a]
            m.set_tuning(fs, as_)
            _say(f"[shapes] {sc.name} candidate {i}: {m.tuning()['fwd_lanes']} / {m.tuning()['adj_lanes']} "
                 f"x {m.tuning()['adj_rays']}")
            p, dth, dsg = _gpu_run(m, sc, K)
            assert np.abs(p - ref.p).max() <= TOL_P, (sc.name, i)
            assert _grad_rel(dth, tb_ref) <= TOL_G, (sc.name, i)
            assert _grad_rel(dsg, sb_ref) <= TOL_G, (sc.name, i)
        m.close()


def test_autotune_keeps_parity(oracle, RayMRF):
    sc = _long_ray_scenes()[0]
    K = 4
    ref, tb_ref, sb_ref = _reference(oracle, sc, K)
    m = RayMRF()
    m.build(sc)
    _gpu_run(m, sc, K)
    t = m.autotune(reps=2)
    _say(f"[autotune] {sc.name}: {t['fwd_lanes']} / {t['adj_lanes']} x {t['adj_rays']}")
    assert all(0 <= s < n for s, n in zip(t["fwd_sel"], t["fwd_candidates"]))
    p, dth, dsg = _gpu_run(m, sc, K)
    assert np.abs(p - ref.p).max() <= TOL_P
    assert _grad_rel(dth, tb_ref) <= TOL_G
    assert _grad_rel(dsg, sb_ref) <= TOL_G
    m.close()
