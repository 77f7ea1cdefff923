"""GPU parity of per-keyframe averaged messages (Sec. IV-A) against the FP64
oracle's or_infer_keyframe_avg on the same seeded scenes: the rays of one
keyframe crossing a voxel send it their chord-length-weighted average, and a
ray's incoming message leaves out its own keyframe.

Bars: marginals within 1e-4; the last sweep's ray -> voxel messages within
2e-4 (1 + |ell*|) plus 1e-6 of the largest |g| on the ray up to the edge (the
log-likelihood magnitudes its FP32 recurrences carry); the last sweep's voxel
-> ray messages within 1e-4 (1 + |lam*|) plus 1e-6 of |theta| and the summed
|average| of the other keyframes into the voxel (the terms it adds)."""
import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_P = 1e-4


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def RayMRF():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2006_03512_amd.mrf import RayMRF as R
    return R


def _two_c4_keyframes():
    sc = S.make_c4()
    return S.Scene(sc.name, sc.depth[:2].copy(), sc.T_wc[:2].copy(), sc.intr, sc.grid, sc.solids,
                   sc.params, sc.sigma_table, sc.prior, sc.sweeps)


def _scenes(name):
    if name == "batch":
        scs = [S.make_fd(), S.random_scene(2), S.make_c1()]
        for x in scs[1:]:   # one set of build parameters and tables per batch
            x.params, x.sigma_table = scs[0].params, scs[0].sigma_table
        return scs
    if name == "c4kf2":
        return [_two_c4_keyframes()]
    if name.startswith("rand"):
        return [S.random_scene(int(name[4:]))]
    return [S.make(name)]


def _running_max_abs(G, x):
    """Per edge: max |x| over the edges of its ray up to and including it."""
    out = np.abs(x).copy()
    lens = np.diff(G.row_ptr)
    nz = lens > 0
    starts = G.row_ptr[:-1][nz]
    ln = lens[nz]
    for j in range(1, int(ln.max()) if ln.size else 0):
        at = starts[ln > j] + j
        out[at] = np.maximum(out[at - 1], out[at])
    return out


def _pair_code(G, key):
    """One int64 per edge naming its (voxel, keyframe) pair, and the keyframe
    count (a 1-D unique over these codes is much faster than one over rows)."""
    nk = int(key.max()) + 1 if key.size else 1
    return G.col.astype(np.int64) * nk + key.astype(np.int64), nk


def _others(G, key, w, ell, theta):
    """Per edge: |theta| plus the summed |average| of the OTHER keyframes into
    its voxel (from the oracle's last-sweep messages)."""
    code, nk = _pair_code(G, key)
    uniq, inv = np.unique(code, return_inverse=True)
    inv = inv.reshape(-1)
    sw = np.bincount(inv, weights=w)
    sm = np.bincount(inv, weights=w * ell)
    avg = np.abs(sm / sw)
    per_voxel = np.abs(theta) + np.bincount(uniq // nk, weights=avg, minlength=theta.size)
    return per_voxel[G.col] - avg[inv]


def _plain_shapes(m):
    """Per ray class, the candidate of one 64-lane wave per ray (the plain
    schedule's untuned shape; the only candidate where no such shape exists)."""
    t0 = m.tuning()
    sel = []
    for q, n in enumerate(t0["fwd_candidates"]):
        pick = 0
        for i in range(n):
            trial = list(t0["fwd_sel"])
            trial[q] = i
            m.set_tuning(fwd_sel=trial)
            if m.tuning()["fwd_lanes"][q] == 64:
                pick = i
                break
        sel.append(pick)
    m.set_tuning(fwd_sel=t0["fwd_sel"])
    return sel


CASES = ["c1", "fd", "rand2", "c2", "batch", "c4kf2"]


@pytest.mark.parametrize("name", CASES)
def test_keyframe_average_matches_oracle(oracle, RayMRF, name):
    scs = _scenes(name)
    K = 3 if name == "batch" else scs[0].sweeps
    _say(f"[keyframe average] {name}: oracle")
    G = oracle.build_graph(scs)
    key, w = oracle.edge_keyframes_and_lengths(G, scs)
    th = np.concatenate([s.prior_logit() for s in scs]).astype(np.float64)
    sig = scs[0].sigma_table
    ref = oracle.infer_keyframe_average(G, th, sig, K, key, w)
    ref_prev = oracle.infer_keyframe_average(G, th, sig, K - 1, key, w) if K > 1 else None
    _say(f"[keyframe average] {name}: GPU ({G.n_edges} edges, {K} sweeps)")
    m = RayMRF()
    st = m.build(scs, keyframe_average=True)
    npairs = np.unique(_pair_code(G, key)[0]).size
    assert st.n_keyframe_pairs == npairs
    m.infer_keyframe_avg(torch.from_numpy(th.astype(np.float32)).cuda(),
                         torch.from_numpy(sig.astype(np.float32)).cuda(), K)
    p, L = m.marginals()
    e = m.export_edges()
    p = p.cpu().numpy().astype(np.float64)
    lam = e["lam"].cpu().numpy().astype(np.float64)
    ell = e["ell"].cpu().numpy().astype(np.float64)
    m.close()
    ep = np.abs(p - ref.p)
    _say(f"  pairs {npairs}; marginals max |p - p*| = {ep.max():.2e}")
    assert np.all(np.isfinite(p)) and ep.max() <= TOL_P
    # last sweep's ray messages
    bl = 2e-4 * (1.0 + np.abs(ref.ell)) + 1e-6 * _running_max_abs(G, ref.g)
    rl = np.abs(ell - ref.ell) / bl
    _say(f"  ell: max err / bound {rl.max():.3f}")
    assert rl.max() <= 1.0
    # last sweep's voxel -> ray messages (the keyframe's message)
    others = _others(G, key, w, ref_prev.ell, th) if ref_prev is not None else np.abs(th[G.col])
    bm = 1e-4 * (1.0 + np.abs(ref.lam)) + 1e-6 * others
    rm = np.abs(lam - ref.lam) / bm
    inf = np.abs(ref.lam) < 10
    _say(f"  lam: max err / bound {rm.max():.3f}; informative edges {int(inf.sum())}, "
         f"max |lam - lam*| there {np.abs(lam - ref.lam)[inf].max() if inf.any() else 0:.3e}")
    assert rm.max() <= 1.0


def test_keyframe_average_single_keyframe_keeps_prior(RayMRF):
    """One keyframe: every voxel -> ray message is the prior in every sweep,
    so the messages after 1 and after 6 sweeps are identical."""
    sc = S.make_c1()
    m = RayMRF()
    m.build(sc, keyframe_average=True)
    th = torch.from_numpy(sc.prior_logit()).cuda()
    sig = torch.from_numpy(sc.sigma_table.astype(np.float32)).cuda()
    m.infer_keyframe_avg(th, sig, 1)
    e1 = m.export_edges()
    m.infer_keyframe_avg(th, sig, 6)
    e6 = m.export_edges()
    assert torch.equal(e1["ell"], e6["ell"]) and torch.equal(e1["lam"], e6["lam"])
    np.testing.assert_array_equal(e6["lam"].cpu().numpy(),
                                  sc.prior_logit()[m.export_incidence()["col"].cpu().numpy()])
    m.close()


def test_keyframe_average_needs_the_build_flag_and_checkpoints_for_a_reverse_pass(RayMRF):
    from paper_2006_03512_amd._lib import MRF_ESTATE, MRFError
    sc = S.make_fd()
    m = RayMRF()
    m.build(sc)
    th = torch.from_numpy(sc.prior_logit()).cuda()
    sig = torch.from_numpy(sc.sigma_table.astype(np.float32)).cuda()
    with pytest.raises(MRFError) as ei:
        m.infer_keyframe_avg(th, sig, 2)
    assert ei.value.code == MRF_ESTATE
    m.build(sc, keyframe_average=True)
    m.infer_keyframe_avg(th, sig, 2)
    with pytest.raises(MRFError) as ei:
        m.backward(torch.zeros_like(th))
    assert ei.value.code == MRF_ESTATE
    # a plain inference on the same build still runs and differentiates
    m.infer(th, sig, 2, keep_checkpoints=True)
    dp, ds = m.backward(torch.zeros_like(th))
    assert torch.all(dp == 0) and torch.all(ds == 0)
    m.close()


def test_keyframe_average_graph_and_plain_schedules_agree(RayMRF):
    """The plain schedule (eager, per-frame launches, one wave per ray) and
    the captured graph with the same launch shapes give identical results."""
    sc = S.make_fd()
    m = RayMRF()
    m.build(sc, keyframe_average=True)
    th = torch.from_numpy(sc.prior_logit()).cuda()
    sig = torch.from_numpy(sc.sigma_table.astype(np.float32)).cuda()
    m.set_schedule("plain")
    m.infer_keyframe_avg(th, sig, 4)
    a = m.marginals()[1].clone()
    m.set_tuning(fwd_sel=_plain_shapes(m))
    m.set_schedule("graph")
    m.infer_keyframe_avg(th, sig, 4)
    b = m.marginals()[1].clone()
    assert torch.equal(a, b)
    m.close()
