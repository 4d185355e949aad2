"""Host-side checks of the C ABI: the library loads, exports every declared symbol, and
validates arguments before launching anything (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "trips.h")


def _lib():
    import paper_2401_06003_amd as tp
    if not os.path.exists(tp.LIB_PATH):
        pytest.skip("libtrips.so not built")
    return tp, tp.lib()


def test_exports_every_declared_symbol():
    tp, L = _lib()
    names = set(re.findall(r"\b(trips_[a-z_]+)\s*\(", open(HEADER).read()))
    assert len(names) >= 11
    for name in sorted(names):
        assert hasattr(L, name), name


def _cam(W=1920, H=1080):
    import scenes
    return scenes.camera([[1, 0, 0], [0, 1, 0], [0, 0, 1]], (0, 0, 3), W, H)


def test_layer_layout_and_sizes():
    tp, L = _lib()
    dims, offs = tp.layer_layout(_cam(), 8)
    assert dims[0] == (1920, 1080) and dims[7] == (15, 9)
    assert offs[-1] == 2764845
    cams = (tp.Camera * 1)(tp.make_camera(_cam()))
    ws, sv = ctypes.c_size_t(), ctypes.c_size_t()
    st = L.trips_buffer_sizes(ctypes.byref(tp.make_config(8, 4)), cams, 1, 2_000_000, None,
                              ctypes.byref(ws), ctypes.byref(sv))
    assert st == 0 and ws.value > 0 and sv.value > 0
    assert sv.value % 256 == 0 and ws.value % 256 == 0


@pytest.mark.parametrize("cfg,views,n,tune,code", [
    ((0, 16, 0.25, 4), 1, 10, None, -1),     # no layers
    ((13, 16, 0.25, 4), 1, 10, None, -1),    # too many layers
    ((5, 8, 0.25, 4), 1, 10, None, -5),      # list clamp other than 16
    ((5, 16, 0.25, 6), 1, 10, None, -5),     # descriptor width not built
    ((5, 16, 1.5, 4), 1, 10, None, -1),      # eps out of range
    ((5, 16, 0.25, 4), 0, 10, None, -1),     # no views
    ((5, 16, 0.25, 4), 17, 10, None, -1),    # too many views
    ((5, 16, 0.25, 4), 1, -1, None, -1),     # negative point count
    ((5, 16, 0.25, 4), 1, 10, (12, 0, 0), -1),   # tile width not a power of two
    ((5, 16, 0.25, 4), 1, 10, (16, 100, 0), -1),  # points per block too small
])
def test_invalid_arguments(cfg, views, n, tune, code):
    tp, L = _lib()
    cams = (tp.Camera * 17)(*[tp.make_camera(_cam(64, 48)) for _ in range(17)])
    t = tp.make_tuning(*tune) if tune else None
    ws, sv = ctypes.c_size_t(), ctypes.c_size_t()
    st = L.trips_buffer_sizes(ctypes.byref(tp.make_config(*cfg[:1], cfg[3], cfg[2], cfg[1])),
                              cams, views, n, ctypes.byref(t) if t else None, ctypes.byref(ws),
                              ctypes.byref(sv))
    assert st == code


PX = 1024 * 768


@pytest.mark.parametrize("n, item", [(1, 8192), (PX, 8192), (PX + 1, 16384), (2 * PX, 16384),
                                     (2 * PX + 1, 32768), (4 * PX, 32768), (10 * PX, 32768)])
def test_default_item_size_follows_density(n, item):
    """The default work-item size is 8192 entries up to one point per pixel of the largest
    view (1024x768 here; the smaller second view does not count), doubled for each doubling
    of the density, up to 32768: the buffers equal those of that explicit size."""
    tp, L = _lib()
    cams = (tp.Camera * 2)(tp.make_camera(_cam(1024, 768)), tp.make_camera(_cam(512, 384)))
    cfg = tp.make_config(5, 4)
    sizes = []
    for t in (None, tp.make_tuning(0, 0, item)):
        ws, sv = ctypes.c_size_t(), ctypes.c_size_t()
        assert L.trips_buffer_sizes(ctypes.byref(cfg), cams, 2, n, ctypes.byref(t) if t else None,
                                    ctypes.byref(ws), ctypes.byref(sv)) == 0
        sizes.append((ws.value, sv.value))
    assert sizes[0] == sizes[1]
    if item < 32768 and n >= PX:  # and differ from the next size up (the check has teeth)
        ws, sv = ctypes.c_size_t(), ctypes.c_size_t()
        up = tp.make_tuning(0, 0, 2 * item)
        assert L.trips_buffer_sizes(ctypes.byref(cfg), cams, 2, n, ctypes.byref(up),
                                    ctypes.byref(ws), ctypes.byref(sv)) == 0
        assert (ws.value, sv.value) != sizes[0]


def test_inclusion_flag_sizes_and_range():
    tp, L = _lib()
    cams = (tp.Camera * 1)(tp.make_camera(_cam(64, 48)))
    sizes = []
    for flag in (0, 1):
        ws, sv = ctypes.c_size_t(), ctypes.c_size_t()
        cfg = tp.make_config(5, 4, include_coarser=flag)
        assert L.trips_buffer_sizes(ctypes.byref(cfg), cams, 1, 1000, None, ctypes.byref(ws),
                                    ctypes.byref(sv)) == 0
        sizes.append((ws.value, sv.value))
    # 4 x 3 + 2 x 2 + 1 + 1 + 1 = 19 tiles of 16x16 over the 64x48 pyramid of 5 layers;
    # inclusion keeps 16 keys, gammas and a count per texel and two (1 + D)-float tables, and
    # drops the per-texel word of kept slots of the fine tiles (it has no fine tiles)
    tiles = 19
    assert sizes[1][1] - sizes[0][1] >= tiles * 256 * (16 * 12 + 4 - 4)
    assert sizes[1][0] > sizes[0][0] and sizes[1][0] >= tiles * 256 * 16 * 5 * 4 * 2
    bad = tp.make_config(5, 4)
    bad.include_coarser = 2
    ws, sv = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.trips_buffer_sizes(ctypes.byref(bad), cams, 1, 1000, None, ctypes.byref(ws),
                                ctypes.byref(sv)) == -1


def test_bad_camera_rejected():
    tp, L = _lib()
    c = _cam(64, 48)
    c["znear"] = 0.0
    cams = (tp.Camera * 1)(tp.make_camera(c))
    ws, sv = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.trips_buffer_sizes(ctypes.byref(tp.make_config(5, 4)), cams, 1, 10, None,
                                ctypes.byref(ws), ctypes.byref(sv)) == -1


def test_forward_validates_before_launch():
    """Every failing check returns before any launch, so these run without a GPU."""
    tp, L = _lib()
    cfg = tp.make_config(5, 4)
    cams = (tp.Camera * 1)(tp.make_camera(_cam(64, 48)))
    ws, sv = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.trips_buffer_sizes(ctypes.byref(cfg), cams, 1, 100, None, ctypes.byref(ws),
                                ctypes.byref(sv)) == 0
    fake = 1 << 20  # aligned, never dereferenced: every call below fails validation first
    pts = tp.Points(fake, fake, fake, fake, fake, fake, 100)
    null_pts = tp.Points(0, 0, 0, 0, 0, 0, 100)
    f = L.trips_forward
    # null point arrays
    assert f(ctypes.byref(cfg), ctypes.byref(null_pts), cams, 1, None, fake, fake, sv.value, fake,
             ws.value, None, None) == -1
    # saved / workspace too small
    assert f(ctypes.byref(cfg), ctypes.byref(pts), cams, 1, None, fake, fake, sv.value - 256, fake,
             ws.value, None, None) == -2
    assert f(ctypes.byref(cfg), ctypes.byref(pts), cams, 1, None, fake, fake, sv.value, fake,
             ws.value - 256, None, None) == -2
    # misaligned saved buffer
    assert f(ctypes.byref(cfg), ctypes.byref(pts), cams, 1, None, fake, fake + 8, sv.value, fake,
             ws.value, None, None) == -1
    # misaligned background (optional arguments are validated too)
    ext = tp.Extras(fake + 4, None, None, None, None)
    assert f(ctypes.byref(cfg), ctypes.byref(pts), cams, 1, None, fake, fake, sv.value, fake,
             ws.value, ctypes.byref(ext), None) == -1
    # point count differs from the one the buffers were sized for is still validated per call
    b = L.trips_backward
    assert b(ctypes.byref(cfg), ctypes.byref(pts), cams, 1, None, 0, fake, sv.value, fake, ws.value,
             fake, fake, fake, fake, fake, fake, None, None) == -1   # null grad_pyramid
    ext = tp.Extras(None, None, None, fake + 4, None)  # misaligned grad_background
    assert b(ctypes.byref(cfg), ctypes.byref(pts), cams, 1, None, fake, fake, sv.value, fake,
             ws.value, fake, fake, fake, fake, fake, fake, ctypes.byref(ext), None) == -1
    assert L.trips_status_string(-3) == b"problem exceeds 32-bit fragment indexing"


def test_autotune_validates_before_launch():
    tp, L = _lib()
    cfg = tp.make_config(5, 4)
    cams = (tp.Camera * 1)(tp.make_camera(_cam(64, 48)))
    fake = 1 << 20
    pts = tp.Points(fake, fake, fake, fake, fake, fake, 100)
    best = tp.Tuning()
    ms = (ctypes.c_float * 2)()
    bad = (tp.Tuning * 2)(tp.make_tuning(16), tp.make_tuning(12))  # second tile width invalid
    st = L.trips_autotune(ctypes.byref(cfg), ctypes.byref(pts), cams, 1, bad, 2, 1, fake, fake,
                          1 << 30, fake, 1 << 30, fake, fake, fake, fake, fake, fake, fake,
                          ctypes.byref(best), ms, None)
    assert st == -1
    assert L.trips_autotune(ctypes.byref(cfg), ctypes.byref(pts), cams, 1, bad, 0, 1, fake, fake,
                            1 << 30, fake, 1 << 30, fake, fake, fake, fake, fake, fake, fake,
                            ctypes.byref(best), ms, None) == -1


def test_view_with_too_many_tiles_is_unsupported():
    """The binning passes keep a 16-bit counter per tile of one view in LDS (at most 32768
    tiles): 3840x2160 with 16x16 tiles over 8 layers has 43,301 and is refused before any
    launch, as is 3600x1800 (34,116); 3200x1600 (26,704) is accepted."""
    tp, L = _lib()
    ws, sv = ctypes.c_size_t(), ctypes.c_size_t()
    cfg = tp.make_config(8, 4)
    for (W, H), code in (((3840, 2160), -5), ((3200, 1600), 0), ((3600, 1800), -5)):
        cams = (tp.Camera * 1)(tp.make_camera(_cam(W, H)))
        assert L.trips_buffer_sizes(ctypes.byref(cfg), cams, 1, 1000, None, ctypes.byref(ws),
                                    ctypes.byref(sv)) == code, (W, H)
    cams = (tp.Camera * 1)(tp.make_camera(_cam(3840, 2160)))
    fake = 1 << 20
    pts = tp.Points(fake, fake, fake, fake, fake, fake, 1000)
    assert L.trips_forward(ctypes.byref(cfg), ctypes.byref(pts), cams, 1, None, fake, fake,
                           1 << 40, fake, 1 << 40, None, None) == -5


def _dec_cfg(tp, nl=4, D=4, out_dim=3, W=64, H=48):
    return tp.DecoderConfig(nl, D, out_dim, W, H)


def test_decoder_sizes():
    tp, L = _lib()
    L = tp._declib()
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.trips_decoder_sizes(ctypes.byref(_dec_cfg(tp, 8, 4, 3, 1920, 1080)),
                                 ctypes.byref(pb), ctypes.byref(wb)) == 0
    # block outputs of layers 1..7 in binary16: 32 channels of every texel below layer 0
    below = sum((-(-1920 // (1 << l))) * (-(-1080 // (1 << l))) for l in range(1, 8))
    assert below * 64 <= wb.value <= below * 64 + 7 * 256
    # packed kernels: (9 + 2) steps x 4 KB per layer but the coarsest (2 steps), plus biases
    assert pb.value >= 7 * 11 * 4096 + 2 * 4096 + 8 * 256


@pytest.mark.parametrize("cfg,code", [
    ((0, 4, 3, 64, 48), -1),    # no layers
    ((13, 4, 3, 64, 48), -1),   # too many layers
    ((4, 6, 3, 64, 48), -5),    # channel count not built
    ((4, 4, 0, 64, 48), -1),    # no output channels
    ((4, 4, 9, 64, 48), -1),    # too many output channels
    ((4, 4, 3, 0, 48), -1),     # empty view
])
def test_decoder_invalid_config(cfg, code):
    tp, L = _lib()
    L = tp._declib()
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.trips_decoder_sizes(ctypes.byref(tp.DecoderConfig(*cfg)), ctypes.byref(pb),
                                 ctypes.byref(wb)) == code


def test_decoder_calls_validate_before_launching():
    """Bad pointers, sizes and layer indices are refused on the host (nothing is launched,
    so no device is needed)."""
    tp, L = _lib()
    L = tp._declib()
    cfg = _dec_cfg(tp)
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    L.trips_decoder_sizes(ctypes.byref(cfg), ctypes.byref(pb), ctypes.byref(wb))
    fake = ctypes.c_void_p(1 << 20)  # aligned, never dereferenced: validation fails first
    null = ctypes.c_void_p(0)
    assert L.trips_decoder_pack(ctypes.byref(cfg), ctypes.byref(tp.DecoderWeights()), fake,
                                pb.value, null) == -1  # missing kernels
    assert L.trips_decoder_forward(ctypes.byref(cfg), fake, pb.value - 1, fake, fake, fake,
                                   wb.value, null) == -2  # packed buffer too small
    assert L.trips_decoder_forward(ctypes.byref(cfg), fake, pb.value, fake, fake, fake,
                                   wb.value - 1, null) == -2  # workspace too small
    assert L.trips_decoder_forward(ctypes.byref(cfg), fake, pb.value, null, fake, fake,
                                   wb.value, null) == -1  # no pyramid
    assert L.trips_decoder_block(ctypes.byref(cfg), fake, pb.value, 4, fake, fake, fake, null,
                                 null) == -1  # layer out of range
    assert L.trips_decoder_block(ctypes.byref(cfg), fake, pb.value, 1, fake, null, fake, null,
                                 null) == -1  # a layer below the coarsest needs its input
    assert L.trips_decoder_block(ctypes.byref(cfg), fake, pb.value, 3, fake, null, fake, fake,
                                 null) == -1  # both outputs given


def test_noalloc_forward_limits():
    """trips_forward_noalloc refuses, on the host and before anything is launched, a problem
    whose forward scratch exceeds the library's static array (8M points at 1920x1080 need
    about 0.8 GB), and takes no workspace argument at all."""
    tp, L = _lib()
    cams = (tp.Camera * 1)(tp.make_camera(_cam()))
    cfg = tp.make_config(8, 4)
    fake = 1 << 20  # aligned, never dereferenced: the size check comes first
    n = 8_000_000
    pts = tp.Points(fake, fake, fake, fake, fake, fake, n)
    ws, sv = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.trips_buffer_sizes(ctypes.byref(cfg), cams, 1, n, None, ctypes.byref(ws),
                                ctypes.byref(sv)) == 0
    st = L.trips_forward_noalloc(ctypes.byref(cfg), ctypes.byref(pts), cams, 1, None,
                                 ctypes.c_void_p(fake), ctypes.c_void_p(fake), sv.value, None,
                                 ctypes.c_void_p(0))
    assert st == -2
    st = L.trips_forward_noalloc(ctypes.byref(cfg), ctypes.byref(pts), cams, 1, None,
                                 ctypes.c_void_p(fake), ctypes.c_void_p(fake), sv.value - 1,
                                 None, ctypes.c_void_p(0))
    assert st == -2  # saved buffer too small
    st = L.trips_forward_noalloc(ctypes.byref(cfg), None, cams, 1, None, ctypes.c_void_p(fake),
                                 ctypes.c_void_p(fake), sv.value, None, ctypes.c_void_p(0))
    assert st == -1
