"""GPU forward parity through the C ABI against the CPU oracle.

Fragment lists (per-texel list lengths, kept point ids and their order) must be bit-exact;
the blended pyramid must be within 1e-5 relative per element."""
import numpy as np
import pytest

import scenes
from gpu_util import PARAMS, assert_lists, assert_pyramid, check_forward, gpu_forward
from oracle import oracle

pytestmark = pytest.mark.gpu


def _tune(tile_w=16, ppb=0, item=0):
    import paper_2401_06003_amd as tp
    return tp.make_tuning(tile_w, ppb, item)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("tile_w", [8, 16, 32, 64])
def test_small_scenes(gpu, seed, tile_w):
    sc = scenes.random_small(100 + seed, n=600, W=97, H=61, nlayers=5, s_lo=0.3, s_hi=24.0)
    check_forward(sc, gpu, _tune(tile_w))


@pytest.mark.parametrize("item", [256, 512])
def test_heavy_lists_split_into_items(gpu, item):
    """Long lists: bins are cut into several work items and their partial top-16s merged."""
    sc = scenes.random_small(7, n=6000, W=40, H=30, nlayers=4, s_lo=2.0, s_hi=12.0)
    res, r, _ = check_forward(sc, gpu, _tune(16, 256, item))
    assert res[0][1].max() > 200
    st = r.stats()
    assert st["items"] > st["bins"]


def test_depth_ties_break_by_index(gpu):
    sc = scenes.random_small(3, n=800, W=48, H=40, nlayers=4, depth_ties=True)
    check_forward(sc, gpu)


def test_unit_cube_4096(gpu):
    """4096 points in the unit cube, 256x256, 5 layers (the CPU-sized workload)."""
    sc = scenes.unit_cube(1)
    res, r, _ = check_forward(sc, gpu)
    assert res[0][1].sum() > 20000


def test_unit_cube_4096_small_launch_shape(gpu):
    """The same workload at the launch shape the autotuner picks for it: 8x32 tiles, 512-point
    binning blocks (eight blocks) and 256-entry work items, so the heavy coarse tiles are cut
    into many items whose partial lists are merged."""
    sc = scenes.unit_cube(1)
    res, r, _ = check_forward(sc, gpu, _tune(8, 512, 256))
    st = r.stats()
    assert st["items"] > st["bins"]


def test_descriptor_width_8(gpu):
    sc = scenes.unit_cube(5, n=2000, W=120, H=90, nlayers=5, D=8)
    check_forward(sc, gpu)


def test_points_per_block_and_ragged_blocks(gpu):
    sc = scenes.unit_cube(6, n=3001, W=100, H=77, nlayers=5)
    check_forward(sc, gpu, _tune(16, 300, 1024))


def test_culled_and_nonfinite_points(gpu):
    sc = scenes.random_small(9, n=300, W=64, H=48, nlayers=4)
    p = sc["points"]
    p["z"][:20] = -1.0          # behind the camera
    p["z"][20:30] = 0.005       # in front of the camera but closer than znear
    p["x"][30:35] = np.nan
    p["sw"][35:40] = np.inf
    p["sw"][40:45] = 0.0        # zero size
    check_forward(sc, gpu)


def test_no_points(gpu):
    sc = scenes.random_small(1, n=0, W=33, H=17, nlayers=3)
    res, _, _ = gpu_forward(sc, gpu)
    assert np.all(res[0][0] == 0) and np.all(res[0][1] == 0) and np.all(res[0][2] == -1)


def test_single_layer_and_deep_pyramid(gpu):
    for nl in (1, 2, 12):
        sc = scenes.random_small(11, n=400, W=70, H=50, nlayers=nl, s_lo=0.2, s_hi=3000.0)
        check_forward(sc, gpu)


def test_rotated_cameras_several_views(gpu):
    sc = scenes.multiview_scene(4, n=20000, views=5, nlayers=6)
    check_forward(sc, gpu)


def test_run_twice_bitwise(gpu):
    sc = scenes.unit_cube(2, n=3000, W=128, H=96)
    a, _, _ = gpu_forward(sc, gpu)
    b, _, _ = gpu_forward(sc, gpu)
    for k in range(3):
        assert np.array_equal(a[0][k], b[0][k])


@pytest.mark.parametrize("item", [512, 1024])
def test_spatially_ordered_points(gpu, item):
    """A cluster scene whose points are in Morton order (consecutive points crowd the same
    texels): every list is compared, with work items small enough that heavy tiles are cut
    into several, whose entries the forward takes as interleaved blocks."""
    sc = scenes.morton_sorted(scenes.cluster_scene(5, n=120_000, W=480, H=270, nlayers=6,
                                                   s_hi=64.0))
    res, r, _ = check_forward(sc, gpu, _tune(16, 0, item))
    entries, _ = r.tile_stats()
    assert (entries > item).sum() > 4  # tiles cut into several items


def test_cluster_scene_full_size_sampled(gpu):
    """2M points, 1920x1080, 8 layers: every texel's list and kept ids are compared on a
    sample of texels from every layer (the oracle evaluates only those texels)."""
    sc = scenes.cluster_scene(2)
    cam, nl = sc["cams"][0], sc["nlayers"]
    res, r, _ = gpu_forward(sc, gpu)
    pyr_g, cnt_g, ids_g = res[0]
    P = len(cnt_g)
    rng = np.random.default_rng(0)
    dims = oracle.layer_dims(cam["W"], cam["H"], nl)
    base = np.cumsum([0] + [w * h for w, h in dims])
    sample = []
    for L in range(nl):
        size = base[L + 1] - base[L]
        sample.append(base[L] + rng.choice(size, min(size, 400), replace=False))
    sample = np.concatenate(sample)
    mask = np.zeros(P, dtype=np.uint8)
    mask[sample] = 1
    pyr, counts, ids = oracle.forward(sc["points"], cam, nl, mask=mask)
    assert_lists(cnt_g[sample], ids_g[sample], counts[sample], ids[sample], "sampled")
    assert_pyramid(pyr_g[sample], pyr[sample], "sampled")
    assert counts[sample].max() > 1000
