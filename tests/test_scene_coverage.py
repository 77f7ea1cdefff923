"""CPU: the scenes of the launch-shape parity test give work to every tile
class from 64 to 640 steps (tiles of 4x4 rays are classed by their longest
ray; the capacities are the library's, as mrf_get_tuning reports them)."""
import numpy as np

from paper_2006_03512_amd import scenes as S

TILE_CLASS_CAPS = [16, 64, 128, 192, 256, 320, 384, 512, 640, 768, 1024, 1536, 2048]


def _tile_lengths(G, sc):
    lens = np.diff(G.row_ptr).reshape(sc.n_frames, sc.intr.height, sc.intr.width)
    out = []
    for f in range(sc.n_frames):
        for ty in range(0, sc.intr.height, 4):
            for tx in range(0, sc.intr.width, 4):
                out.append(lens[f, ty:ty + 4, tx:tx + 4].max())
    out = np.array(out)
    return out[out > 0]


def test_long_ray_scenes_reach_the_lds_classes(oracle):
    caps_reached = set()
    scs = [S.random_scene(21, grid=(400, 400, 24), voxel=0.01, n_frames=2),
           S.random_scene(22, grid=(320, 320, 40), voxel=0.0125, n_frames=2),
           S.random_scene(23, grid=(480, 480, 20), voxel=0.01, n_frames=2)]
    for sc in scs:
        tl = _tile_lengths(oracle.build_graph(sc), sc)
        caps_reached |= {TILE_CLASS_CAPS[int(np.searchsorted(TILE_CLASS_CAPS, n))] for n in tl}
    assert {64, 128, 192, 256, 320, 384, 512, 640} <= caps_reached, sorted(caps_reached)
