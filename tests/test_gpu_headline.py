"""GPU parity at the benchmark's geometry: the first two keyframes of the
30-keyframe room batch (full 640 x 480 frames into the 250 x 250 x 150 grid at
0.02 m, 1.2e8 edges), K = 8 sweeps with checkpoints and the reverse pass,
against the FP64 oracle on the same frames.

This is where voxels receive thousands of ray messages and near-camera rays
send messages of 1e6 log-odds, so the voxel -> ray message of Eq.
node_to_factor (the prior plus every other ray's message) is a small number
left over from large ones.  The bar for it is set on the message itself and
on the terms it actually sums (the prior and the OTHER rays' messages), never
on the receiving ray's own message, which the sum must not depend on:

  |lam - lam*| <= 1e-4 (1 + |lam*|) + 1e-6 (|theta| + sum over the other
                                            rays' |ell*|)

on every edge whose |lam*| < 10 (an informative message).  Prior and
sigma-table gradients by the relative 1e-3 rule (norm per group, and per entry
against |g*| + max |g*|).

Marginals: within 1e-4 of the oracle, widened on each voxel by ten times how
far the FP64 oracle's own marginal moves when its messages are stored at
single precision (FP64 arithmetic, every lambda and ell rounded to float32
after each phase, two rounding patterns): 1e-4 + 10 * spread_v.  A handful of
voxels at this geometry receive a message that is an O(1) difference of
log-likelihoods of magnitude 1e5 (rays whose every likelier voxel is believed
empty by the other rays' messages of 1e9), so a float32 ulp of the messages
the difference is taken from already moves the exact answer by more than
1e-4; everywhere else spread_v is below 1e-6 and the bar is 1e-4 itself."""
import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_P = 1e-4
TOL_G = 1e-3


def _say(msg):
    print(msg, flush=True)


def _grad_check(g, ref):
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    ent = np.abs(g - ref) / (np.abs(ref) + np.abs(ref).max())
    return rel, ent.max()


@pytest.fixture(scope="module")
def two_keyframes(oracle):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    _say("[headline] generating the 30-keyframe batch, keeping keyframes 0 and 1")
    sc = S.make_c4()
    sub = S.Scene(sc.name, sc.depth[:2].copy(), sc.T_wc[:2].copy(), sc.intr, sc.grid, sc.solids,
                  sc.params, sc.sigma_table, sc.prior, sc.sweeps)
    K = sub.sweeps
    G = oracle.build_graph(sub)
    th = sub.prior_logit().astype(np.float64)
    y = sub.occupancy().astype(np.float64)
    _say(f"[headline] oracle: {G.n_edges} edges, {K} sweeps with history")
    ref = oracle.infer(G, th, sub.sigma_table, K, keep_history=True)
    ref_prev = oracle.infer(G, th, sub.sigma_table, K - 1)   # the ray messages lambda^(K) sums
    spread = np.zeros(G.n_voxels)
    for mode in (1, 2):
        spread = np.maximum(spread, np.abs(oracle.infer_f32_storage(G, th, sub.sigma_table, K, mode).p - ref.p))
    tb_ref, sb_ref, _ = oracle.backward(G, ref, oracle.bce_logit_grad(ref.L, y), sub.sigma_table)
    _say("[headline] oracle done; GPU build, infer, reverse pass")
    from paper_2006_03512_amd.mrf import RayMRF
    m = RayMRF()
    m.build(sub)
    thd = torch.from_numpy(sub.prior_logit()).cuda()
    sig = torch.from_numpy(sub.sigma_table.astype(np.float32)).cuda()
    m.infer(thd, sig, K, keep_checkpoints=True)
    p, L = m.marginals()
    e = m.export_edges()
    lam = e["lam"].cpu().numpy().astype(np.float64)
    ell = e["ell"].cpu().numpy().astype(np.float64)
    dth, dsg = m.backward((p - torch.from_numpy(y.astype(np.float32)).cuda()) / p.numel())
    out = {"p": p.cpu().numpy(), "lam": lam, "ell": ell, "dtheta": dth.cpu().numpy(), "dsigma": dsg.cpu().numpy()}
    torch.cuda.synchronize()
    m.close()
    yield G, th, ref, ref_prev, tb_ref, sb_ref, out, spread


def test_headline_marginals(two_keyframes):
    G, th, ref, _, _, _, out, spread = two_keyframes
    err = np.abs(out["p"] - ref.p)
    over = np.where(err > TOL_P)[0]
    _say(f"  marginals: max |p - p*| = {err.max():.2e}; {over.size} voxels above {TOL_P:g}, "
         f"{int((spread > TOL_P).sum())} voxels whose oracle spread under float32 storage is above it")
    for v in over[:10]:
        _say(f"    voxel {v}: |p - p*| = {err[v]:.3e}, p* = {ref.p[v]:.6f}, oracle spread {spread[v]:.3e}")
    well = spread < 1e-6
    _say(f"  voxels with spread < 1e-6: {int(well.sum())}, max |p - p*| there {err[well].max():.2e}")
    assert np.all(np.isfinite(out["p"]))
    assert np.all(err <= TOL_P + 10.0 * spread)
    assert err[well].max() <= TOL_P


def test_headline_informative_messages(two_keyframes):
    """Last sweep's voxel -> ray messages on informative edges, bounded on
    |lam*| and the terms they sum, not on the receiving ray's own message."""
    G, th, ref, ref_prev, _, _, out, _ = two_keyframes
    lam_star = ref.lam
    own = np.abs(ref_prev.ell)
    mag = np.abs(th).copy()
    np.add.at(mag, G.col, own)
    others = mag[G.col] - own      # |theta| + sum of the other rays' |ell*| into the voxel
    inf = np.abs(lam_star) < 10.0
    err = np.abs(out["lam"] - lam_star)
    plain = err / (1e-4 * (1.0 + np.abs(lam_star)))
    bound = 1e-4 * (1.0 + np.abs(lam_star)) + 1e-6 * others
    r = err / bound
    worst = int(np.argmax(np.where(inf, err, -1.0)))
    _say(f"  {int(inf.sum())} informative edges; worst |lam - lam*| = {err[worst]:.3e} at lam* = "
         f"{lam_star[worst]:.4f} (own |ell*| = {own[worst]:.3e}, others {others[worst]:.3e}); "
         f"max err / 1e-4(1+|lam*|) = {plain[inf].max():.3f}, max err / bound = {r[inf].max():.3f}; "
         f"own |ell*| up to {own[inf].max():.3e}")
    assert inf.sum() > 1000000
    assert r[inf].max() <= 1.0


def test_headline_ray_messages(two_keyframes):
    """Last sweep's ray -> voxel messages (Eqs. pos, neg) on edges whose
    |ell*| < 10: within 2e-4 (1 + |ell*|) plus 1e-6 of the largest |g| among
    the voxels up to and including the edge on its ray (the log-likelihoods the
    prefix recurrence of the message has summed)."""
    G, _, ref, _, _, _, out, _ = two_keyframes
    lens = np.diff(G.row_ptr)
    nz = lens > 0
    ag = np.abs(ref.g)
    # running maximum of |g| along each ray, one step index at a time
    pre = ag.copy()
    starts = G.row_ptr[:-1][nz]
    ln = lens[nz]
    for j in range(1, int(ln.max())):
        at = starts[ln > j] + j
        pre[at] = np.maximum(pre[at - 1], ag[at])
    ell_star = ref.ell
    inf = np.abs(ell_star) < 10.0
    err = np.abs(out["ell"] - ell_star)
    bound = 2e-4 * (1.0 + np.abs(ell_star)) + 1e-6 * pre
    r = err / bound
    _say(f"  {int(inf.sum())} informative ray messages; max err {err[inf].max():.3e}, "
         f"max err / bound {r[inf].max():.3f}; all edges: max err / bound {r.max():.3f}")
    assert r[inf].max() <= 1.0


def test_headline_gradients(two_keyframes):
    _, _, _, _, tb_ref, sb_ref, out, _ = two_keyframes
    r1, e1 = _grad_check(out["dtheta"], tb_ref)
    r2, e2 = _grad_check(out["dsigma"], sb_ref)
    _say(f"  theta rel {r1:.2e} entry {e1:.2e}; sigma rel {r2:.2e} entry {e2:.2e}")
    assert r1 <= TOL_G and e1 <= TOL_G
    assert r2 <= TOL_G and e2 <= TOL_G
