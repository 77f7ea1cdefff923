"""A batch of more than 2^32 edge slots at the benchmark's geometry: two copies
of a 36-keyframe room (640 x 480 frames into the 250 x 250 x 150 grid at
0.02 m, about 2.2e9 slots each) in one build, which forms two groups of
scenes, so the second scene's slots all lie above 2^32.  The oracle cannot
run BP at this size; the checks are properties that hold at any size: each
scene of the batch gives the marginals of that scene built alone (the scenes
are independent MRFs), both copies give the same marginals, and the batch's
counts are twice a copy's."""
import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

K = 2


def _say(msg):
    print(msg, flush=True)


def test_two_groups_above_2e32_slots():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2006_03512_amd.mrf import RayMRF
    _say("[groups] generating a 36-keyframe room")
    sc = S.make_c4(n_frames=36)
    theta1 = torch.from_numpy(sc.prior_logit()).cuda()
    sigma = torch.from_numpy(sc.sigma_table.astype(np.float32)).cuda()
    m = RayMRF()
    st1 = m.build(sc)
    _say(f"[groups] one copy: {st1.n_slots} slots, {st1.n_edges} edges, {st1.n_slot_groups} group")
    assert st1.n_slot_groups == 1 and 2 * st1.n_slots >= (1 << 32)
    m.infer(theta1, sigma, K)
    alone = m.marginals()[1].cpu().numpy()
    m.close()
    torch.cuda.empty_cache()
    m = RayMRF()
    st2 = m.build([sc, sc])
    _say(f"[groups] two copies: {st2.n_slots} slots, {st2.n_edges} edges, {st2.n_slot_groups} groups")
    assert st2.n_slot_groups == 2
    assert st2.n_slots == 2 * st1.n_slots and st2.n_edges == 2 * st1.n_edges
    assert st2.n_rays == 2 * st1.n_rays
    m.infer(torch.cat([theta1, theta1]), sigma, K)
    both = m.marginals()[1].cpu().numpy()
    m.close()
    V = sc.grid.n_voxels
    a, b = both[:V], both[V:]
    np.testing.assert_array_equal(a, b)
    pa = np.exp(-np.logaddexp(0.0, -alone.astype(np.float64)))   # sigmoid without overflow
    pb = np.exp(-np.logaddexp(0.0, -b.astype(np.float64)))
    err = np.abs(pa - pb).max()
    _say(f"[groups] second copy (slots above 2^32) against the room alone: max |dp| = {err:.2e}")
    assert err <= 1e-6
