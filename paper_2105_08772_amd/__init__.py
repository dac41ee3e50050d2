"""Python binding of the C ABI declared in include/lbm_sc.h.

Argument marshalling only: every step of the computation runs in the HIP library
liblbm_sc.so (built in-tree for gfx950 by paper_2105_08772_amd.build). Loading fails loudly if
the library is missing; there is no CPU fallback.

The functions carry the C names. Host arrays are numpy float64 in the canonical layout
f[i][z][y][x] (shape (19, nz, ny, nx)).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_sc.so")

LBM_SC_OK, LBM_SC_EINVAL, LBM_SC_ENOMEM, LBM_SC_EDEVICE, LBM_SC_EUNSTABLE = 0, -1, -2, -3, -4
LBM_SC_PSI_EXP, LBM_SC_PSI_ONEMINUS = 0, 1
LBM_SC_DROPLET, LBM_SC_BUBBLE, LBM_SC_SLAB, LBM_SC_FROM_HOST = 0, 1, 2, 3
LBM_SC_FP64, LBM_SC_FP32_SHIFTED, LBM_SC_FP32_SHIFTED_MATH64 = 0, 1, 2

_i32, _i64, _u64, _f64, _vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
                               ctypes.c_void_p)


class LbmScConfig(ctypes.Structure):
    _fields_ = [("nx", _i32), ("ny", _i32), ("nz", _i32), ("psi", _i32), ("geom", _i32),
                ("prec", _i32), ("slab_axis", _i32), ("packed_rows", _i32), ("tau", _f64),
                ("g_over_gc", _f64), ("radius", _f64), ("width", _f64), ("slab_thickness", _f64),
                ("n_in", _f64), ("n_out", _f64), ("noise_amp", _f64), ("seed", _u64),
                ("rho_ref", _f64), ("stream", _vp)]


class LbmScObs(ctypes.Structure):
    _fields_ = [("step", _i64), ("mass", _f64), ("mass0", _f64), ("mom", _f64 * 3),
                ("com", _f64 * 3), ("n_center", _f64), ("n_far", _f64), ("P_in", _f64),
                ("P_out", _f64), ("dP", _f64), ("C", _f64), ("R_s", _f64), ("sigma_s", _f64),
                ("R_e", _f64), ("sigma0_flat", _f64), ("pn_spread", _f64), ("du_l1", _f64),
                ("du_max", _f64), ("n_min", _f64), ("n_max", _f64), ("finite", _i32),
                ("has_du", _i32)]

    def to_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if name in ("mom", "com") else v
        return out


class LbmScInfo(ctypes.Structure):
    _fields_ = [("G", _f64), ("Gc", _f64), ("n_in", _f64), ("n_out", _f64), ("rho_ref", _f64),
                ("nodes", _i64), ("device_bytes", _i64), ("bytes_per_step", _i64),
                ("block_x", _i32), ("block_y", _i32), ("z_chunk", _i32), ("reserved", _i32)]

    def to_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class LbmScLaunch(ctypes.Structure):
    _fields_ = [("rows", _i32), ("z_chunk", _i32), ("xcd_remap", _i32), ("prefetch", _i32),
                ("waves", _i32), ("tile_x", _i32), ("graph_steps", _i32),
                ("steps_per_pass", _i32)]

    def to_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class LbmScGroupLaunch(ctypes.Structure):
    _fields_ = [("rows", _i32), ("z_chunk", _i32), ("xcd_remap", _i32), ("prefetch", _i32),
                ("persistent", _i32), ("workers", _i32), ("graph_steps", _i32), ("waves", _i32),
                ("tile_x", _i32), ("items_per_cu", _i32), ("steps_per_pass", _i32)]

    def to_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class LbmScError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm_sc error {code}: {msg}")
        self.code = code


EXPORTS = ("lbm_sc_create", "lbm_sc_step", "lbm_sc_sync", "lbm_sc_observables",
           "lbm_sc_get_populations", "lbm_sc_set_populations", "lbm_sc_set_launch",
           "lbm_sc_get_launch", "lbm_sc_stream_copy", "lbm_sc_get_info", "lbm_sc_destroy",
           "lbm_sc_last_error", "lbm_sc_gc", "lbm_sc_coexistence", "lbm_sc_group_create",
           "lbm_sc_group_set", "lbm_sc_group_step", "lbm_sc_group_set_launch",
           "lbm_sc_group_get_launch", "lbm_sc_group_info", "lbm_sc_group_destroy",
           "lbm_sc_device_bytes", "lbm_sc_create_with_buffers", "lbm_sc_population_bytes",
           "lbm_sc_set_step", "lbm_sc_step_boxes_noalloc")

_lib = None


def load():
    """Load liblbm_sc.so. torch is imported first so that the library binds to the same HIP
    runtime as torch (both name libamdhip64.so.7)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (shares its HIP runtime with the library)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    L.lbm_sc_create.argtypes = [P(LbmScConfig), P(_vp)]
    L.lbm_sc_create_with_buffers.argtypes = [P(LbmScConfig), _vp, _vp, ctypes.c_size_t, P(_vp)]
    L.lbm_sc_population_bytes.argtypes = [P(LbmScConfig)]
    L.lbm_sc_population_bytes.restype = _i64
    L.lbm_sc_step.argtypes = [_vp, _i64]
    L.lbm_sc_sync.argtypes = [_vp]
    L.lbm_sc_observables.argtypes = [_vp, P(LbmScObs), P(_f64), ctypes.c_size_t]
    L.lbm_sc_get_populations.argtypes = [_vp, P(_f64), ctypes.c_size_t]
    L.lbm_sc_set_populations.argtypes = [_vp, P(_f64), ctypes.c_size_t]
    L.lbm_sc_set_step.argtypes = [_vp, _i64]
    L.lbm_sc_set_launch.argtypes = [_vp, P(LbmScLaunch)]
    L.lbm_sc_get_launch.argtypes = [_vp, P(LbmScLaunch)]
    L.lbm_sc_stream_copy.argtypes = [_vp, _vp, ctypes.c_size_t, _i32, _vp]
    L.lbm_sc_get_info.argtypes = [_vp, P(LbmScInfo)]
    L.lbm_sc_destroy.argtypes = [_vp]
    L.lbm_sc_destroy.restype = None
    L.lbm_sc_last_error.argtypes = []
    L.lbm_sc_last_error.restype = ctypes.c_char_p
    L.lbm_sc_gc.argtypes = [_i32]
    L.lbm_sc_gc.restype = _f64
    L.lbm_sc_coexistence.argtypes = [_i32, _f64, P(_f64), P(_f64), P(_f64)]
    L.lbm_sc_group_create.argtypes = [_vp, P(_vp)]
    L.lbm_sc_group_set.argtypes = [_vp, P(_vp), _i32]
    L.lbm_sc_group_step.argtypes = [_vp, _i64]
    L.lbm_sc_group_set_launch.argtypes = [_vp, P(LbmScGroupLaunch)]
    L.lbm_sc_group_get_launch.argtypes = [_vp, P(LbmScGroupLaunch)]
    L.lbm_sc_group_info.argtypes = [_vp, P(_i32), P(_i64), P(_i64), P(_i64)]
    L.lbm_sc_group_destroy.argtypes = [_vp]
    L.lbm_sc_group_destroy.restype = None
    L.lbm_sc_step_boxes_noalloc.argtypes = [P(_vp), _i32, _i64, P(LbmScGroupLaunch)]
    L.lbm_sc_device_bytes.argtypes = [P(LbmScConfig)]
    L.lbm_sc_device_bytes.restype = _i64
    for name in EXPORTS:
        if name not in ("lbm_sc_destroy", "lbm_sc_last_error", "lbm_sc_gc",
                        "lbm_sc_group_destroy", "lbm_sc_device_bytes",
                        "lbm_sc_population_bytes"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc):
    if rc != LBM_SC_OK:
        raise LbmScError(rc, lbm_sc_last_error())


def config(nx, ny=None, nz=None, *, psi=LBM_SC_PSI_EXP, geom=LBM_SC_DROPLET, prec=LBM_SC_FP64,
           slab_axis=2, tau=1.0, g_over_gc=1.3, radius=0.0, width=2.0, slab_thickness=0.0,
           n_in=0.0, n_out=0.0, noise_amp=0.0, seed=0, rho_ref=0.0, stream=None, packed_rows=0):
    """Build an lbm_sc_config (fields as documented in include/lbm_sc.h)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return LbmScConfig(nx, ny, nz, psi, geom, prec, slab_axis, packed_rows, tau, g_over_gc,
                       radius, width,
                       slab_thickness, n_in, n_out, noise_amp, seed & (2**64 - 1), rho_ref,
                       stream)


def lbm_sc_last_error():
    return load().lbm_sc_last_error().decode()


def lbm_sc_gc(psi):
    return load().lbm_sc_gc(psi)


def lbm_sc_coexistence(psi, g_over_gc):
    ng, nl, p0 = _f64(), _f64(), _f64()
    _check(load().lbm_sc_coexistence(psi, g_over_gc, ctypes.byref(ng), ctypes.byref(nl),
                                      ctypes.byref(p0)))
    return ng.value, nl.value, p0.value


def lbm_sc_device_bytes(cfg):
    v = load().lbm_sc_device_bytes(ctypes.byref(cfg))
    if v < 0:
        raise LbmScError(v, lbm_sc_last_error())
    return v


def lbm_sc_create(cfg):
    h = _vp()
    _check(load().lbm_sc_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h


def lbm_sc_population_bytes(cfg):
    v = load().lbm_sc_population_bytes(ctypes.byref(cfg))
    if v < 0:
        raise LbmScError(v, lbm_sc_last_error())
    return v


def lbm_sc_create_with_buffers(cfg, a, b, nbytes):
    """a, b: device addresses (ints) of the caller's two population buffers."""
    h = _vp()
    _check(load().lbm_sc_create_with_buffers(ctypes.byref(cfg), _vp(a), _vp(b), int(nbytes),
                                             ctypes.byref(h)))
    return h


def lbm_sc_step(h, nsteps):
    _check(load().lbm_sc_step(h, int(nsteps)))


def lbm_sc_sync(h):
    _check(load().lbm_sc_sync(h))


def lbm_sc_observables(h, profile_len=None, raise_unstable=True):
    """Returns (obs dict, profile array (4, L) or None). profile_len is L (None: no profile)."""
    o = LbmScObs()
    prof = None
    if profile_len:
        prof = np.zeros(4 * profile_len)
        rc = load().lbm_sc_observables(h, ctypes.byref(o), prof.ctypes.data_as(ctypes.POINTER(_f64)),
                                       prof.size)
        prof = prof.reshape(4, profile_len)
    else:
        rc = load().lbm_sc_observables(h, ctypes.byref(o), None, 0)
    if rc == LBM_SC_EUNSTABLE and not raise_unstable:
        return o.to_dict(), prof
    _check(rc)
    return o.to_dict(), prof


def lbm_sc_get_populations(h, dims):
    nx, ny, nz = dims
    f = np.empty((19, nz, ny, nx))
    _check(load().lbm_sc_get_populations(h, f.ctypes.data_as(ctypes.POINTER(_f64)), f.size))
    return f


def lbm_sc_set_populations(h, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    _check(load().lbm_sc_set_populations(h, f.ctypes.data_as(ctypes.POINTER(_f64)), f.size))


def lbm_sc_set_step(h, step):
    _check(load().lbm_sc_set_step(h, int(step)))


def lbm_sc_set_launch(h, rows, z_chunk, xcd_remap=1, prefetch=0, waves=4, tile_x=64,
                      graph_steps=64, steps_per_pass=1):
    l = LbmScLaunch(rows, z_chunk, xcd_remap, prefetch, waves, tile_x, graph_steps,
                    steps_per_pass)
    _check(load().lbm_sc_set_launch(h, ctypes.byref(l)))


def lbm_sc_get_launch(h):
    l = LbmScLaunch()
    _check(load().lbm_sc_get_launch(h, ctypes.byref(l)))
    return l.to_dict()


def lbm_sc_stream_copy(src_ptr, dst_ptr, nbytes, stream=None, lane_bytes=4):
    """Streaming copy of nbytes between device addresses (measurement helper); lane_bytes: 4, 8
    or 16 bytes moved by each lane per access."""
    _check(load().lbm_sc_stream_copy(src_ptr, dst_ptr, nbytes, int(lane_bytes), stream))


def lbm_sc_get_info(h):
    i = LbmScInfo()
    _check(load().lbm_sc_get_info(h, ctypes.byref(i)))
    return i.to_dict()


def lbm_sc_destroy(h):
    if h is not None and h.value:
        load().lbm_sc_destroy(h)


class Box:
    """Owner of one lbm_sc handle (destroyed with the object). `buffers`: optionally two device
    tensors (e.g. torch.empty(lbm_sc_population_bytes(cfg), dtype=torch.uint8, device="cuda"))
    that hold the populations in place of library allocations; the box keeps them alive."""

    def __init__(self, cfg, buffers=None):
        self.cfg = cfg
        self.dims = (cfg.nx, cfg.ny, cfg.nz)
        self.buffers = buffers
        if buffers is None:
            self.h = lbm_sc_create(cfg)
        else:
            import torch
            a, b = buffers
            for t in (a, b):
                if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
                    raise ValueError("buffers must be two contiguous device tensors")
            nbytes = min(a.numel() * a.element_size(), b.numel() * b.element_size())
            # work already queued on torch's stream for this memory (a caching allocator hands
            # out blocks whose last use may still be running) ends before the box's stream uses it
            torch.cuda.current_stream(a.device).synchronize()
            self.h = lbm_sc_create_with_buffers(cfg, a.data_ptr(), b.data_ptr(), nbytes)

    def step(self, n):
        lbm_sc_step(self.h, n)

    def sync(self):
        lbm_sc_sync(self.h)

    def profile_len(self):
        if self.cfg.geom == LBM_SC_SLAB:
            return self.dims[self.cfg.slab_axis]
        return self.cfg.nx

    def observables(self, profile=True, raise_unstable=True):
        return lbm_sc_observables(self.h, self.profile_len() if profile else None, raise_unstable)

    def get(self):
        return lbm_sc_get_populations(self.h, self.dims)

    def set(self, f):
        lbm_sc_set_populations(self.h, f)

    def set_step(self, step):
        lbm_sc_set_step(self.h, step)

    def set_launch(self, rows, z_chunk, xcd_remap=1, prefetch=0, waves=4, tile_x=64,
                   graph_steps=64, steps_per_pass=1):
        lbm_sc_set_launch(self.h, rows, z_chunk, xcd_remap, prefetch, waves, tile_x, graph_steps,
                          steps_per_pass)

    def launch(self):
        return lbm_sc_get_launch(self.h)

    def info(self):
        return lbm_sc_get_info(self.h)

    def close(self):
        if self.h is not None:
            lbm_sc_destroy(self.h)   # waits for the box's stream: the buffers are free after it
            self.h = None
        self.buffers = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def lbm_sc_group_create(stream):
    g = _vp()
    _check(load().lbm_sc_group_create(stream, ctypes.byref(g)))
    return g


def lbm_sc_group_set(g, handles):
    arr = (_vp * max(len(handles), 1))(*[h.value for h in handles])
    _check(load().lbm_sc_group_set(g, arr, len(handles)))


def lbm_sc_group_step(g, nsteps):
    _check(load().lbm_sc_group_step(g, int(nsteps)))


def lbm_sc_group_get_launch(g):
    l = LbmScGroupLaunch()
    _check(load().lbm_sc_group_get_launch(g, ctypes.byref(l)))
    return l.to_dict()


def lbm_sc_group_set_launch(g, **kw):
    cur = lbm_sc_group_get_launch(g)
    cur.update(kw)
    l = LbmScGroupLaunch(**cur)
    _check(load().lbm_sc_group_set_launch(g, ctypes.byref(l)))


def lbm_sc_group_info(g):
    nb, it, nn, bb = _i32(), _i64(), _i64(), _i64()
    _check(load().lbm_sc_group_info(g, ctypes.byref(nb), ctypes.byref(it), ctypes.byref(nn),
                                    ctypes.byref(bb)))
    return dict(nbox=nb.value, items=it.value, nodes=nn.value, bytes_per_step=bb.value)


def lbm_sc_group_destroy(g):
    if g is not None and g.value:
        load().lbm_sc_group_destroy(g)


LBM_SC_NOALLOC_MAX_BOXES = 1024
LBM_SC_OBS_WORKSPACE_BYTES_PER_NODE = 40


def lbm_sc_step_boxes_noalloc(handles, nsteps, **launch):
    """nsteps steps of the boxes (handles) with one multi-box launch per step and no device
    allocation; `launch` holds the fields of lbm_sc_group_launch."""
    l = LbmScGroupLaunch(**launch)
    arr = (_vp * max(len(handles), 1))(*[h.value for h in handles])
    _check(load().lbm_sc_step_boxes_noalloc(arr, len(handles), int(nsteps), ctypes.byref(l)))


class Group:
    """Owner of one lbm_sc_group handle. `stream` is a hipStream_t (int); the boxes added must
    have been created with the same stream."""

    def __init__(self, stream):
        self.stream = stream
        self.g = lbm_sc_group_create(stream)
        self.boxes = []

    def set(self, boxes):
        lbm_sc_group_set(self.g, [b.h for b in boxes])
        self.boxes = list(boxes)

    def step(self, n):
        lbm_sc_group_step(self.g, n)

    def set_launch(self, **kw):
        lbm_sc_group_set_launch(self.g, **kw)

    def launch(self):
        return lbm_sc_group_get_launch(self.g)

    def info(self):
        return lbm_sc_group_info(self.g)

    def close(self):
        if self.g is not None:
            lbm_sc_group_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
