"""Trilinear point splatting (TRIPS, Sec. 3.1-3.2) on MI355X: thin Python binding.

Every step of the renderer runs in the HIP kernels of libtrips.so behind the C ABI in
include/trips.h; this module only marshals arguments.  PyTorch provides device memory
and the stream.  If the library is not built, importing works but every call raises.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtrips.so")
KEEP = 16
MAX_VIEWS = 16

c_float, c_int32, c_int64, c_void_p, c_size_t = (ctypes.c_float, ctypes.c_int32, ctypes.c_int64,
                                                  ctypes.c_void_p, ctypes.c_size_t)


class Camera(ctypes.Structure):
    _fields_ = [("R", c_float * 9), ("t", c_float * 3), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("width", c_int32), ("height", c_int32),
                ("znear", c_float)]


class Config(ctypes.Structure):
    _fields_ = [("num_layers", c_int32), ("max_list", c_int32), ("eps", c_float),
                ("desc_dim", c_int32), ("include_coarser", c_int32)]


class Points(ctypes.Structure):
    _fields_ = [("x", c_void_p), ("y", c_void_p), ("z", c_void_p), ("size_w", c_void_p),
                ("opacity", c_void_p), ("desc", c_void_p), ("n", c_int64)]


class Extras(ctypes.Structure):
    """Optional arguments (trips_extras): background, coverage, their gradients, camera grads."""
    _fields_ = [("background", c_void_p), ("alpha_out", c_void_p), ("grad_alpha", c_void_p),
                ("grad_background", c_void_p), ("grad_camera", c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_w", c_int32), ("points_per_block", c_int32), ("item_entries", c_int32)]


STATUS = {0: "ok", -1: "invalid argument", -2: "workspace or saved buffer too small",
          -3: "capacity", -4: "HIP error", -5: "unsupported"}


class TripsError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s failed: %s (%d)" % (what, STATUS.get(status, "?"), status))


_lib = None


def lib():
    """The loaded libtrips.so; raises if it was not built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libtrips.so is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.trips_layer_layout.argtypes = [P(Camera), P(Config), P(c_int32), P(c_int64)]
        L.trips_buffer_sizes.argtypes = [P(Config), P(Camera), c_int32, c_int64, P(Tuning),
                                         P(c_size_t), P(c_size_t)]
        L.trips_forward.argtypes = [P(Config), P(Points), P(Camera), c_int32, P(Tuning), c_void_p,
                                    c_void_p, c_size_t, c_void_p, c_size_t, c_void_p, c_void_p]
        L.trips_forward_noalloc.argtypes = [P(Config), P(Points), P(Camera), c_int32, P(Tuning),
                                            c_void_p, c_void_p, c_size_t, c_void_p, c_void_p]
        L.trips_forward_noalloc.restype = c_int32
        L.trips_backward.argtypes = [P(Config), P(Points), P(Camera), c_int32, P(Tuning), c_void_p,
                                     c_void_p, c_size_t, c_void_p, c_size_t] + [c_void_p] * 8
        L.trips_export_fragments.argtypes = [P(Config), P(Camera), c_int32, P(Tuning), c_void_p,
                                             c_size_t, c_void_p, c_void_p, c_void_p]
        L.trips_forward_stats.argtypes = [P(Config), P(Camera), c_int32, P(Tuning), c_void_p,
                                          c_size_t, P(c_int64), c_void_p]
        L.trips_tile_stats.argtypes = [P(Config), P(Camera), c_int32, P(Tuning), c_void_p,
                                       c_size_t, c_void_p, c_void_p, c_void_p]
        L.trips_status_string.argtypes = [c_int32]
        L.trips_status_string.restype = ctypes.c_char_p
        L.trips_last_hip_error.restype = c_int32
        L.trips_timing_enable.argtypes = [c_int32]
        L.trips_timing_enable.restype = c_int32
        L.trips_timing_read.argtypes = [P(c_float), P(c_int32)]
        L.trips_timing_read.restype = c_int32
        L.trips_stage_name.argtypes = [c_int32]
        L.trips_stage_name.restype = ctypes.c_char_p
        L.trips_autotune.argtypes = ([P(Config), P(Points), P(Camera), c_int32, P(Tuning), c_int32,
                                      c_int32, c_void_p, c_void_p, c_size_t, c_void_p, c_size_t]
                                     + [c_void_p] * 7 + [P(Tuning), P(c_float), c_void_p])
        L.trips_autotune.restype = c_int32
        L.trips_plan_create.argtypes = ([P(Config), P(Points), P(Camera), c_int32, P(Tuning),
                                         c_void_p, c_void_p, c_size_t, c_void_p, c_size_t]
                                        + [c_void_p] * 9 + [P(c_void_p)])
        L.trips_plan_launch.argtypes = [c_void_p, c_int32, c_void_p]
        L.trips_plan_destroy.argtypes = [c_void_p]
        for name in ("trips_layer_layout", "trips_buffer_sizes", "trips_forward", "trips_backward",
                     "trips_export_fragments", "trips_forward_stats", "trips_tile_stats",
                     "trips_plan_create", "trips_plan_launch"):
            getattr(L, name).restype = c_int32
        L.trips_plan_destroy.restype = None
        _lib = L
    return _lib


def _check(status, what):
    if status != 0:
        if status == -4:
            what = "%s (hip error %d)" % (what, lib().trips_last_hip_error())
        raise TripsError(status, what)


def make_camera(cam):
    """Camera struct from a dict {R (9), t (3), fx, fy, cx, cy, W, H, znear}."""
    c = Camera()
    R = [float(v) for v in list(cam["R"]).__iter__()] if not hasattr(cam["R"], "reshape") else \
        [float(v) for v in cam["R"].reshape(-1)]
    t = [float(v) for v in (cam["t"].reshape(-1) if hasattr(cam["t"], "reshape") else cam["t"])]
    c.R[:] = R
    c.t[:] = t
    c.fx, c.fy, c.cx, c.cy = float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"])
    c.width, c.height = int(cam["W"]), int(cam["H"])
    c.znear = float(cam.get("znear", 0.01))
    return c


def make_config(num_layers, desc_dim, eps=0.25, max_list=KEEP, include_coarser=False):
    return Config(int(num_layers), int(max_list), float(eps), int(desc_dim),
                  int(bool(include_coarser)))


def make_tuning(tile_w=0, points_per_block=0, item_entries=0):
    return Tuning(int(tile_w), int(points_per_block), int(item_entries))


def layer_layout(cam, num_layers):
    """[(W_L, H_L)] and texel offsets of one view."""
    cfg = make_config(num_layers, 4)
    dims = (c_int32 * (2 * num_layers))()
    offs = (c_int64 * (num_layers + 1))()
    _check(lib().trips_layer_layout(ctypes.byref(make_camera(cam)), ctypes.byref(cfg), dims, offs),
           "trips_layer_layout")
    return [(dims[2 * L], dims[2 * L + 1]) for L in range(num_layers)], list(offs)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _extras(background=None, alpha_out=None, grad_alpha=None, grad_background=None,
            grad_camera=None):
    """A pointer to a trips_extras struct, or NULL when no field is given."""
    fields = (background, alpha_out, grad_alpha, grad_background, grad_camera)
    if all(f is None for f in fields):
        return None, ctypes.c_void_p(0)
    for f in fields:
        if f is not None and (f.dtype != torch.float32 or not f.is_contiguous()):
            raise ValueError("extra arrays must be contiguous float32")
    e = Extras(*[f.data_ptr() if f is not None else None for f in fields])
    return e, ctypes.c_void_p(ctypes.addressof(e))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _aligned_bytes(nbytes, device):
    """A uint8 tensor of at least nbytes whose data pointer is 256-byte aligned."""
    buf = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + max(int(nbytes), 1)]


class _SavedState:
    """Which forward call last wrote a `saved` buffer (shared by renderers that share it)."""

    def __init__(self):
        self.generation = 0
        self.owner = None


class Renderer:
    """Renders one or more views (different resolutions allowed) of a point cloud.

    Owns the `saved` and `workspace` device buffers (torch tensors) sized by the library.
    include_coarser: coarser-layer inclusion (Sec. 3.6): every texel also blends the
    fragments of the coarser layers' texels that cover it."""

    def __init__(self, cams, num_layers, desc_dim, n_points, eps=0.25, tuning=None,
                 device="cuda", share_buffers_with=None, include_coarser=False):
        if isinstance(cams, dict):
            cams = [cams]
        if not 1 <= len(cams) <= MAX_VIEWS:
            raise ValueError("1..%d views per renderer" % MAX_VIEWS)
        self.cams_py = cams
        self.V = len(cams)
        self.cams = (Camera * self.V)(*[make_camera(c) for c in cams])
        self.cfg = make_config(num_layers, desc_dim, eps, include_coarser=include_coarser)
        self.tune = tuning if tuning is not None else make_tuning()
        self.n = int(n_points)
        self.D = int(desc_dim)
        self.num_layers = int(num_layers)
        ws, sv = c_size_t(), c_size_t()
        _check(lib().trips_buffer_sizes(ctypes.byref(self.cfg), self.cams, self.V, self.n,
                                        ctypes.byref(self.tune), ctypes.byref(ws), ctypes.byref(sv)),
               "trips_buffer_sizes")
        self.ws_bytes, self.saved_bytes = ws.value, sv.value
        self.device = torch.device(device)
        o = share_buffers_with
        if o is not None and o.ws_bytes >= self.ws_bytes and o.saved_bytes >= self.saved_bytes:
            # calls of the two renderers must not overlap on the device (same stream)
            self.workspace, self.saved = o.workspace, o.saved
            self.ws_bytes, self.saved_bytes = o.ws_bytes, o.saved_bytes
            self._saved_state = o._saved_state
        else:
            self.workspace = _aligned_bytes(self.ws_bytes, self.device)
            self.saved = _aligned_bytes(self.saved_bytes, self.device)
            self._saved_state = _SavedState()
        self.layouts = [layer_layout(c, num_layers) for c in cams]
        self.view_texels = [lay[1][-1] for lay in self.layouts]
        self.texels = sum(self.view_texels)

    def pyramid_numel(self):
        return self.texels * self.D

    def _points(self, x, y, z, sw, alpha, desc):
        for t in (x, y, z, sw, alpha, desc):
            if t.dtype != torch.float32 or not t.is_contiguous() or t.device != self.device:
                raise ValueError("point arrays must be contiguous float32 on %s" % self.device)
        if x.numel() != self.n or desc.numel() != self.n * self.D:
            raise ValueError("point count does not match the renderer")
        return Points(x.data_ptr(), y.data_ptr(), z.data_ptr(), sw.data_ptr(), alpha.data_ptr(),
                      desc.data_ptr(), self.n)

    def _texel_array(self, t, per_texel, name):
        if t is not None and t.numel() != self.texels * per_texel:
            raise ValueError("%s must hold %d values per texel" % (name, per_texel))

    def forward(self, x, y, z, sw, alpha, desc, out=None, background=None, alpha_out=None):
        """Flat float32 pyramid: views, then layers, each row-major [H_L][W_L][D].

        background (optional, [P*D]): composited behind the kept fragments with the
        transmittance they leave; alpha_out (optional, [P]) receives the coverage."""
        pts = self._points(x, y, z, sw, alpha, desc)
        if out is None:
            out = torch.empty(self.pyramid_numel(), dtype=torch.float32, device=self.device)
        self._texel_array(background, self.D, "background")
        self._texel_array(alpha_out, 1, "alpha_out")
        keep, ext = _extras(background=background, alpha_out=alpha_out)
        # the saved lists now belong to this call: a backward of an earlier forward that used
        # the same buffer would read them (TripsSplat checks the generation)
        self._saved_state.generation += 1
        self._saved_state.owner = self
        _check(lib().trips_forward(ctypes.byref(self.cfg), ctypes.byref(pts), self.cams, self.V,
                                   ctypes.byref(self.tune), _ptr(out), _ptr(self.saved),
                                   self.saved_bytes, _ptr(self.workspace), self.ws_bytes, ext,
                                   _stream()),
               "trips_forward")
        return out

    def forward_noalloc(self, x, y, z, sw, alpha, desc, out=None, background=None,
                        alpha_out=None):
        """forward() through trips_forward_noalloc: the forward scratch comes from the
        library's static per-GPU array instead of this renderer's workspace (the `out`
        pyramid and the `saved` buffer are still this renderer's)."""
        pts = self._points(x, y, z, sw, alpha, desc)
        if out is None:
            out = torch.empty(self.pyramid_numel(), dtype=torch.float32, device=self.device)
        self._texel_array(background, self.D, "background")
        self._texel_array(alpha_out, 1, "alpha_out")
        keep, ext = _extras(background=background, alpha_out=alpha_out)
        self._saved_state.generation += 1
        self._saved_state.owner = self
        _check(lib().trips_forward_noalloc(ctypes.byref(self.cfg), ctypes.byref(pts), self.cams,
                                           self.V, ctypes.byref(self.tune), _ptr(out),
                                           _ptr(self.saved), self.saved_bytes, ext, _stream()),
               "trips_forward_noalloc")
        return out

    def backward(self, x, y, z, sw, alpha, desc, grad_pyramid, outs=None, background=None,
                 grad_alpha=None, grad_background=None, grad_camera=None):
        """Gradients (x, y, z, sw, alpha, desc) of sum(grad_pyramid * pyramid)
        (+ sum(grad_alpha * coverage) when grad_alpha is given).  background must be the one
        the forward call used; grad_background ([P*D]) and grad_camera ([V, 16]: dR
        row-major, dt, dfx, dfy, dcx, dcy per view) are filled when given."""
        pts = self._points(x, y, z, sw, alpha, desc)
        g = grad_pyramid.contiguous()
        if g.numel() != self.pyramid_numel() or g.dtype != torch.float32:
            raise ValueError("grad_pyramid must be float32 with the pyramid's size")
        self._texel_array(background, self.D, "background")
        self._texel_array(grad_alpha, 1, "grad_alpha")
        self._texel_array(grad_background, self.D, "grad_background")
        if grad_camera is not None and grad_camera.numel() != self.V * 16:
            raise ValueError("grad_camera must hold 16 values per view")
        if outs is None:
            outs = [torch.empty(self.n, dtype=torch.float32, device=self.device) for _ in range(5)]
            outs.append(torch.empty((self.n, self.D), dtype=torch.float32, device=self.device))
        keep, ext = _extras(background=background, grad_alpha=grad_alpha,
                            grad_background=grad_background, grad_camera=grad_camera)
        _check(lib().trips_backward(ctypes.byref(self.cfg), ctypes.byref(pts), self.cams, self.V,
                                    ctypes.byref(self.tune), _ptr(g), _ptr(self.saved),
                                    self.saved_bytes, _ptr(self.workspace), self.ws_bytes,
                                    *[_ptr(o) for o in outs], ext, _stream()),
               "trips_backward")
        return outs

    def export_fragments(self):
        """(counts [P] int32, ids [P, 16] int32) of the last forward call."""
        counts = torch.empty(self.texels, dtype=torch.int32, device=self.device)
        ids = torch.empty((self.texels, KEEP), dtype=torch.int32, device=self.device)
        _check(lib().trips_export_fragments(ctypes.byref(self.cfg), self.cams, self.V,
                                            ctypes.byref(self.tune), _ptr(self.saved),
                                            self.saved_bytes, _ptr(counts), _ptr(ids), _stream()),
               "trips_export_fragments")
        return counts, ids

    def stats(self):
        """{'entries', 'items', 'bins', 'visible'} of the last forward call (synchronises)."""
        st = (c_int64 * 4)()
        _check(lib().trips_forward_stats(ctypes.byref(self.cfg), self.cams, self.V,
                                         ctypes.byref(self.tune), _ptr(self.saved),
                                         self.saved_bytes, st, _stream()), "trips_forward_stats")
        return {"entries": st[0], "items": st[1], "bins": st[2], "visible": st[3]}

    def tile_stats(self):
        """Per-tile (entries, kept fragments) of the last forward call, numpy uint32 arrays in
        bin order (synchronises; for reports)."""
        import numpy as np
        nb = self.stats()["bins"]
        ent = np.zeros(nb, dtype=np.uint32)
        kept = np.zeros(nb, dtype=np.uint32)
        _check(lib().trips_tile_stats(ctypes.byref(self.cfg), self.cams, self.V,
                                      ctypes.byref(self.tune), _ptr(self.saved), self.saved_bytes,
                                      ent.ctypes.data_as(c_void_p), kept.ctypes.data_as(c_void_p),
                                      _stream()), "trips_tile_stats")
        return ent, kept

    def split(self, flat):
        """Per view, per layer [H_L, W_L, D] views of a flat pyramid."""
        out, o = [], 0
        for (dims, _offs) in self.layouts:
            views = []
            for (w, h) in dims:
                views.append(flat[o:o + w * h * self.D].view(h, w, self.D))
                o += w * h * self.D
            out.append(views)
        return out


NUM_STAGES = 14


def timing_enable(on=True):
    """Bracket every kernel of later calls (this thread) with HIP events on its stream."""
    _check(lib().trips_timing_enable(1 if on else 0), "trips_timing_enable")


def timing_read():
    """{stage: (milliseconds summed, launches)} since the last read; waits for the events."""
    ms = (c_float * NUM_STAGES)()
    n = (c_int32 * NUM_STAGES)()
    _check(lib().trips_timing_read(ms, n), "trips_timing_read")
    return {lib().trips_stage_name(k).decode(): (ms[k], n[k]) for k in range(NUM_STAGES)}


class Plan:
    """The batched form captured in a HIP graph: buffers bound once, replayed per launch."""

    def __init__(self, renderer, x, y, z, sw, alpha, desc, pyramid, grad_pyramid=None,
                 grads=None, **extras):
        r = renderer
        self.r = r
        self.keep = (x, y, z, sw, alpha, desc, pyramid, grad_pyramid, grads, extras)
        self._ext_struct, ext = _extras(**extras)
        pts = r._points(x, y, z, sw, alpha, desc)
        g = grads if grads is not None else [None] * 6
        h = c_void_p()
        # capture on a stream of our own (the null stream cannot be captured)
        cap = torch.cuda.Stream(device=r.device)
        cap.wait_stream(torch.cuda.current_stream(r.device))
        st = lib().trips_plan_create(ctypes.byref(r.cfg), ctypes.byref(pts), r.cams, r.V,
                                     ctypes.byref(r.tune), _ptr(pyramid), _ptr(r.saved),
                                     r.saved_bytes, _ptr(r.workspace), r.ws_bytes,
                                     _ptr(grad_pyramid), *[_ptr(t) for t in g], ext,
                                     ctypes.c_void_p(cap.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise TripsError(st, "trips_plan_create (hip error %d)" % lib().trips_last_hip_error())
        self.h = h

    def launch(self, forward=True, backward=False):
        which = (1 if forward else 0) | (2 if backward else 0)
        _check(lib().trips_plan_launch(self.h, which, _stream()), "trips_plan_launch")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.trips_plan_destroy(self.h)
            self.h = None


# Launch shapes tried by default: tile width x points per binning block x entries per item.
DEFAULT_CANDIDATES = [(tw, pb, ie) for tw in (8, 16, 32) for pb in (4096, 8192)
                      for ie in (4096, 8192, 16384)]


def autotune(cams, num_layers, desc_dim, x, y, z, sw, alpha, desc, candidates=None, reps=3,
             cache_path=None, device="cuda"):
    """Pick the fastest launch shape for this workload with the library's autotuner
    (trips_autotune: forward + backward timed with HIP events per candidate).

    Results are cached in a JSON file (cache_path, default $TRIPS_TUNE_CACHE if set) keyed
    by the device name and the workload's shape.  Returns (Tuning, {candidate: ms})."""
    import json
    if isinstance(cams, dict):
        cams = [cams]
    dev = torch.device(device)
    n = int(x.numel())
    cand = [tuple(int(v) for v in c) for c in (candidates or DEFAULT_CANDIDATES)]
    key = json.dumps({"device": torch.cuda.get_device_name(dev), "n": n, "layers": int(num_layers),
                      "D": int(desc_dim), "views": [(int(c["W"]), int(c["H"])) for c in cams],
                      "candidates": cand})
    cache_path = cache_path or os.environ.get("TRIPS_TUNE_CACHE")
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return make_tuning(*cache[key]["best"]), {tuple(k): v for k, v in cache[key]["ms"]}
    cam_arr = (Camera * len(cams))(*[make_camera(c) for c in cams])
    cfg = make_config(num_layers, desc_dim)
    tunes = (Tuning * len(cand))(*[make_tuning(*c) for c in cand])
    ws_max = sv_max = 0
    for k in range(len(cand)):
        ws, sv = c_size_t(), c_size_t()
        _check(lib().trips_buffer_sizes(ctypes.byref(cfg), cam_arr, len(cams), n,
                                        ctypes.byref(tunes[k]), ctypes.byref(ws), ctypes.byref(sv)),
               "trips_buffer_sizes")
        ws_max, sv_max = max(ws_max, ws.value), max(sv_max, sv.value)
    workspace = _aligned_bytes(ws_max, dev)
    saved = _aligned_bytes(sv_max, dev)
    texels = sum(layer_layout(c, num_layers)[1][-1] for c in cams)
    pyr = torch.empty(texels * desc_dim, dtype=torch.float32, device=dev)
    gen = torch.Generator(device=dev).manual_seed(0)
    gpyr = torch.randn(texels * desc_dim, dtype=torch.float32, device=dev, generator=gen)
    grads = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(5)]
    grads.append(torch.empty((n, desc_dim), dtype=torch.float32, device=dev))
    pts = Points(x.data_ptr(), y.data_ptr(), z.data_ptr(), sw.data_ptr(), alpha.data_ptr(),
                 desc.data_ptr(), n)
    best = Tuning()
    ms = (c_float * len(cand))()
    _check(lib().trips_autotune(ctypes.byref(cfg), ctypes.byref(pts), cam_arr, len(cams), tunes,
                                len(cand), int(reps), _ptr(pyr), _ptr(saved), sv_max,
                                _ptr(workspace), ws_max, _ptr(gpyr), *[_ptr(g) for g in grads],
                                ctypes.byref(best), ms, _stream()), "trips_autotune")
    result = {cand[k]: ms[k] for k in range(len(cand))}
    if cache_path:
        cache[key] = {"best": [best.tile_w, best.points_per_block, best.item_entries],
                      "ms": [[list(k), v] for k, v in result.items()]}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best, result


class TripsSplat(torch.autograd.Function):
    """Differentiable render: (x, y, z, sw, alpha, desc) -> flat pyramid."""

    @staticmethod
    def forward(ctx, x, y, z, sw, alpha, desc, renderer):
        args = [t.detach().contiguous() for t in (x, y, z, sw, alpha, desc)]
        out = renderer.forward(*args)
        ctx.renderer = renderer
        ctx.generation = renderer._saved_state.generation
        ctx.save_for_backward(*args)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        r = ctx.renderer
        st = r._saved_state
        if st.generation != ctx.generation:
            raise RuntimeError(
                "TripsSplat.backward: the renderer's saved fragment lists were overwritten by "
                "a later forward call (of this renderer or of one sharing its buffers); run "
                "backward before the next forward, or use one renderer per pending backward")
        grads = r.backward(*ctx.saved_tensors, grad_out)
        return tuple(grads) + (None,)


def render(x, y, z, sw, alpha, desc, renderer):
    """Flat pyramid of `renderer`'s views; differentiable in all six point arrays."""
    return TripsSplat.apply(x, y, z, sw, alpha, desc, renderer)


# ---------------------------------------------------------------------------------------
# Reconstruction network (Sec. 3.3): trips_decoder_* in include/trips.h.

DEC_FEATURES = 32


class DecoderConfig(ctypes.Structure):
    _fields_ = [("num_layers", c_int32), ("desc_dim", c_int32), ("out_dim", c_int32),
                ("width", c_int32), ("height", c_int32)]


class DecoderWeights(ctypes.Structure):
    _fields_ = [("kernel", c_void_p * 12), ("bias", c_void_p * 12), ("out_weight", c_void_p),
                ("out_bias", c_void_p)]


def _declib():
    L = lib()
    if not getattr(L, "_dec_ready", False):
        P = ctypes.POINTER
        L.trips_decoder_sizes.argtypes = [P(DecoderConfig), P(c_size_t), P(c_size_t)]
        L.trips_decoder_pack.argtypes = [P(DecoderConfig), P(DecoderWeights), c_void_p, c_size_t,
                                         c_void_p]
        L.trips_decoder_forward.argtypes = [P(DecoderConfig), c_void_p, c_size_t, c_void_p,
                                            c_void_p, c_void_p, c_size_t, c_void_p]
        L.trips_decoder_block.argtypes = [P(DecoderConfig), c_void_p, c_size_t, c_int32,
                                          c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
        for name in ("trips_decoder_sizes", "trips_decoder_pack", "trips_decoder_forward",
                     "trips_decoder_block", "trips_decoder_last_hip_error"):
            getattr(L, name).restype = c_int32
        L._dec_ready = True
    return L


def _dcheck(status, what):
    if status != 0:
        if status == -4:
            what = "%s (hip error %d)" % (what, _declib().trips_decoder_last_hip_error())
        raise TripsError(status, what)


class Decoder:
    """The reconstruction network of one view size: packs the weights once (device memory
    from torch) and runs the whole network or single blocks.

    weights: {"w": [L] binary16 kernels [3, 3, C_in, 64], "b": [L] float32 [64],
    "wo": float32 [32, out_dim], "bo": float32 [out_dim]} (numpy or torch)."""

    def __init__(self, width, height, num_layers, desc_dim, weights, device="cuda"):
        self.device = torch.device(device)
        out_dim = int(weights["wo"].shape[1])
        self.cfg = DecoderConfig(int(num_layers), int(desc_dim), out_dim, int(width), int(height))
        self.nl, self.D, self.out_dim = int(num_layers), int(desc_dim), out_dim
        pb, wb = c_size_t(), c_size_t()
        _dcheck(_declib().trips_decoder_sizes(ctypes.byref(self.cfg), ctypes.byref(pb),
                                              ctypes.byref(wb)), "trips_decoder_sizes")
        self.packed_bytes, self.ws_bytes = pb.value, wb.value
        self.packed = _aligned_bytes(self.packed_bytes, self.device)
        self.workspace = _aligned_bytes(self.ws_bytes, self.device)
        self.dims = [(-(-int(width) // (1 << L)), -(-int(height) // (1 << L)))
                     for L in range(self.nl)]

        def dev(a, dtype):
            t = torch.as_tensor(a)
            if dtype == torch.float16:
                t = t.to(torch.float16).view(torch.int16)
            else:
                t = t.to(dtype)
            return t.contiguous().to(self.device)

        self._w = [dev(k, torch.float16) for k in weights["w"]]
        self._b = [dev(b, torch.float32) for b in weights["b"]]
        self._wo = dev(weights["wo"], torch.float32)
        self._bo = dev(weights["bo"], torch.float32)
        for L, k in enumerate(self._w):
            cin = self.D if L == self.nl - 1 else self.D + DEC_FEATURES
            if tuple(k.shape) != (3, 3, cin, 2 * DEC_FEATURES):
                raise ValueError("layer %d kernel must be [3, 3, %d, 64]" % (L, cin))
        ws = DecoderWeights()
        for L in range(self.nl):
            ws.kernel[L] = self._w[L].data_ptr()
            ws.bias[L] = self._b[L].data_ptr()
        ws.out_weight, ws.out_bias = self._wo.data_ptr(), self._bo.data_ptr()
        _dcheck(_declib().trips_decoder_pack(ctypes.byref(self.cfg), ctypes.byref(ws),
                                             _ptr(self.packed), self.packed_bytes, _stream()),
                "trips_decoder_pack")

    def forward(self, pyramid, image=None):
        """pyramid: flat float32 (layers in order, [H_L][W_L][D]) -> image [H, W, out_dim]."""
        W, H = self.dims[0]
        if pyramid.dtype != torch.float32 or not pyramid.is_contiguous():
            raise ValueError("pyramid must be contiguous float32")
        if pyramid.numel() != sum(w * h for w, h in self.dims) * self.D:
            raise ValueError("pyramid size does not match the decoder")
        if image is None:
            image = torch.empty((H, W, self.out_dim), dtype=torch.float32, device=self.device)
        _dcheck(_declib().trips_decoder_forward(ctypes.byref(self.cfg), _ptr(self.packed),
                                                self.packed_bytes, _ptr(pyramid), _ptr(image),
                                                _ptr(self.workspace), self.ws_bytes, _stream()),
                "trips_decoder_forward")
        return image

    def block(self, layer, features, coarse=None, final=False):
        """One block: features float32 [H_L, W_L, D]; coarse binary16 [H_L+1, W_L+1, 32] (None
        for the coarsest layer).  Returns the block output (float16 [H_L, W_L, 32]) or, with
        final=True, the output layer applied to it (float32 [H_L, W_L, out_dim])."""
        W, H = self.dims[layer]
        features = features.contiguous()
        if coarse is not None:
            coarse = coarse.contiguous()
        if final:
            out = torch.empty((H, W, self.out_dim), dtype=torch.float32, device=self.device)
            args = (c_void_p(0), _ptr(out))
        else:
            out = torch.empty((H, W, DEC_FEATURES), dtype=torch.float16, device=self.device)
            args = (_ptr(out), c_void_p(0))
        _dcheck(_declib().trips_decoder_block(ctypes.byref(self.cfg), _ptr(self.packed),
                                              self.packed_bytes, int(layer), _ptr(features),
                                              _ptr(coarse), *args, _stream()),
                "trips_decoder_block")
        return out
