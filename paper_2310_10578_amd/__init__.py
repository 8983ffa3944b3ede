"""Python binding of libutd.so, the MI355X smooth-surface UTD field library.

Argument marshalling only: every step of the field evaluation runs in the
library's HIP kernels.  Device buffers are torch tensors on the GPU; the
functions here check shapes and dtypes, allocate outputs with torch and pass
raw pointers and the current HIP stream through the C ABI declared in
``include/utd.h``.  There is no CPU fallback: without the built library or a
GPU every entry point raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libutd.so")

UTD_OK = 0
FLAG_INSIDE, FLAG_CAUSTIC, FLAG_LOS, FLAG_TX_INSIDE = 1, 2, 4, 8
FLAG_INVALID_RX, FLAG_BAD_BODY, FLAG_BAD_FREQ = 16, 32, 64
BAD_RX, BAD_BODY, BAD_FREQ = 1, 2, 4

EXPORTS = ["utd_default_options", "utd_scene_create", "utd_scene_destroy", "utd_scene_triangles",
           "utd_scene_nodes", "utd_smooth_field", "utd_smooth_field_backward", "utd_smooth_field_batched",
           "utd_path_census", "utd_batched_config", "utd_profile_enable", "utd_profile_read", "utd_last_error",
           "utd_path_masks", "utd_input_status", "utd_smooth_field_noalloc", "utd_scene_planes",
           "utd_scene_set_wall_material", "utd_wall_masks", "utd_smooth_field_saved",
           "utd_smooth_field_backward_saved", "utd_forward_state_release"]
KERNELS = ["prep", "occlude", "field", "backward", "reduce", "batched", "walls", "caustic"]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("l_enc", ctypes.c_int), ("bodies_occlude", ctypes.c_int),
                ("lit_branch", ctypes.c_int), ("caustic_guard", ctypes.c_double), ("wall_reflections", ctypes.c_int),
                ("caustic_uniform", ctypes.c_int)]


class WallMaterial(ctypes.Structure):
    _fields_ = [("eps_r", ctypes.c_double), ("sigma", ctypes.c_double), ("thickness", ctypes.c_double),
                ("perfect_conductor", ctypes.c_int)]


class Bodies(ctypes.Structure):
    _fields_ = [("sph", ctypes.c_void_p), ("n_sph", ctypes.c_int64),
                ("cyl", ctypes.c_void_p), ("n_cyl", ctypes.c_int64)]


class Source(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_float * 3), ("dipole", ctypes.c_float * 3), ("amplitude", ctypes.c_double)]


_lib = None


def load_library(path=LIB_PATH):
    """Load libutd.so and declare its signatures (works without a GPU)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libutd.so is not built (%s); run __graft_entry__.build()" % path)
    # One HIP runtime per process: PyTorch bundles its own libamdhip64, so it
    # is loaded first and libutd's dependency resolves to that copy (stream
    # handles and device pointers then belong to the same runtime).  Loading
    # libutd first would bring in a second runtime that hides the GPU from torch.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.utd_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.utd_default_options.restype = None
    lib.utd_scene_create.argtypes = [vp, i64, ctypes.POINTER(vp)]
    lib.utd_scene_create.restype = i32
    lib.utd_scene_destroy.argtypes = [vp]
    lib.utd_scene_destroy.restype = None
    lib.utd_scene_triangles.argtypes = [vp]
    lib.utd_scene_triangles.restype = i64
    lib.utd_scene_nodes.argtypes = [vp]
    lib.utd_scene_nodes.restype = i64
    lib.utd_smooth_field.argtypes = [vp, ctypes.POINTER(Bodies), ctypes.POINTER(Source), vp, i64, vp, i32,
                                     ctypes.POINTER(Options), vp, vp, vp]
    lib.utd_smooth_field.restype = i32
    lib.utd_smooth_field_noalloc.argtypes = lib.utd_smooth_field.argtypes
    lib.utd_smooth_field_noalloc.restype = i32
    lib.utd_smooth_field_backward.argtypes = [vp, ctypes.POINTER(Bodies), ctypes.POINTER(Source), vp, i64, vp, i32,
                                              ctypes.POINTER(Options), vp, vp, vp, vp, vp]
    lib.utd_smooth_field_backward.restype = i32
    lib.utd_smooth_field_saved.argtypes = [vp, ctypes.POINTER(Bodies), ctypes.POINTER(Source), vp, i64, vp, i32,
                                           ctypes.POINTER(Options), vp, vp, ctypes.POINTER(vp), vp]
    lib.utd_smooth_field_saved.restype = i32
    lib.utd_smooth_field_backward_saved.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.utd_smooth_field_backward_saved.restype = i32
    lib.utd_forward_state_release.argtypes = [vp, vp]
    lib.utd_forward_state_release.restype = i32
    lib.utd_smooth_field_batched.argtypes = [vp, i64, vp, vp, i64, vp, vp, i64, ctypes.POINTER(Source), vp, i32,
                                             ctypes.POINTER(Options), vp, vp, vp]
    lib.utd_batched_config.argtypes = [i32, i32]
    lib.utd_batched_config.restype = i32
    lib.utd_smooth_field_batched.restype = i32
    lib.utd_path_census.argtypes = [vp, ctypes.POINTER(Bodies), ctypes.POINTER(Source), vp, i64,
                                    ctypes.POINTER(Options), vp, vp]
    lib.utd_path_census.restype = i32
    lib.utd_path_masks.argtypes = [vp, ctypes.POINTER(Bodies), ctypes.POINTER(Source), vp, i64,
                                   ctypes.POINTER(Options), vp, vp, vp]
    lib.utd_path_masks.restype = i32
    lib.utd_input_status.argtypes = [vp]
    lib.utd_input_status.restype = i32
    lib.utd_scene_planes.argtypes = [vp, vp]
    lib.utd_scene_planes.restype = i64
    lib.utd_scene_set_wall_material.argtypes = [vp, ctypes.POINTER(WallMaterial)]
    lib.utd_scene_set_wall_material.restype = i32
    lib.utd_wall_masks.argtypes = [vp, ctypes.POINTER(Bodies), ctypes.POINTER(Source), vp, i64,
                                   ctypes.POINTER(Options), vp, vp]
    lib.utd_wall_masks.restype = i32
    lib.utd_profile_enable.argtypes = [i32]
    lib.utd_profile_enable.restype = None
    lib.utd_profile_read.argtypes = [vp, vp]
    lib.utd_profile_read.restype = i32
    lib.utd_last_error.argtypes = []
    lib.utd_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


class UTDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("utd status %d: %s" % (status, msg))
        self.status = status


def _check(status):
    if status != UTD_OK:
        raise UTDError(status, load_library().utd_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the UTD library needs a ROCm GPU; none is visible")
    return torch


def _dev(t, dtype, shape_tail, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a GPU torch tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if shape_tail is not None and tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError("%s must have shape [n, %s]" % (name, ", ".join(map(str, shape_tail))))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def make_options(precision=0, l_enc=0, bodies_occlude=True, lit_branch=True, caustic_guard=1e-6,
                 wall_reflections=False, caustic_uniform=False):
    o = Options()
    load_library().utd_default_options(ctypes.byref(o))
    o.precision, o.l_enc = int(precision), int(l_enc)
    o.bodies_occlude, o.lit_branch = int(bool(bodies_occlude)), int(bool(lit_branch))
    o.caustic_guard = float(caustic_guard)
    o.wall_reflections = int(bool(wall_reflections))
    o.caustic_uniform = int(bool(caustic_uniform))
    return o


def make_source(pos, dipole=(0.0, 0.0, 1.0), amplitude=1.0):
    s = Source()
    for a in range(3):
        s.pos[a] = float(pos[a])
        s.dipole[a] = float(dipole[a])
    s.amplitude = float(amplitude)
    return s


class Scene:
    """Occluder triangles (host float32 [n, 3, 3]) and their device BVH."""

    def __init__(self, tri=None):
        import numpy as np
        lib = load_library()
        self._h = ctypes.c_void_p()
        if tri is None:
            arr = np.zeros((0, 3, 3), np.float32)
        else:
            arr = np.ascontiguousarray(tri, dtype=np.float32).reshape(-1, 3, 3)
        self._keep = arr
        _check(lib.utd_scene_create(arr.ctypes.data if arr.size else None, arr.shape[0], ctypes.byref(self._h)))
        self.n_tri = int(lib.utd_scene_triangles(self._h))
        self.n_nodes = int(lib.utd_scene_nodes(self._h))

    @property
    def handle(self):
        return self._h

    def planes(self):
        """Reflecting planes: float64 array [n, 4] of (n_x, n_y, n_z, d)."""
        import numpy as np
        lib = load_library()
        n = int(lib.utd_scene_planes(self._h, None))
        out = np.zeros((n, 4), np.float64)
        if n:
            lib.utd_scene_planes(self._h, out.ctypes.data)
        return out

    def set_wall_material(self, eps_r=3.75, sigma=0.038, thickness=0.10, perfect_conductor=False):
        m = WallMaterial(float(eps_r), float(sigma), float(thickness), int(bool(perfect_conductor)))
        _check(load_library().utd_scene_set_wall_material(self._h, ctypes.byref(m)))

    def close(self):
        if self._h:
            load_library().utd_scene_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _bodies(spheres, cylinders):
    torch = _torch()
    b = Bodies()
    sph = spheres if spheres is not None else torch.zeros((0, 4), dtype=torch.float32, device="cuda")
    cyl = cylinders if cylinders is not None else torch.zeros((0, 5), dtype=torch.float32, device="cuda")
    _dev(sph, torch.float32, (4,), "spheres")
    _dev(cyl, torch.float32, (5,), "cylinders")
    b.sph, b.n_sph = (sph.data_ptr() if sph.numel() else None), sph.shape[0]
    b.cyl, b.n_cyl = (cyl.data_ptr() if cyl.numel() else None), cyl.shape[0]
    return b, (sph, cyl)


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def smooth_field(scene, spheres, cylinders, source, rx, freqs, precision=0, l_enc=0, bodies_occlude=True,
                 lit_branch=True, caustic_guard=1e-6, out=None, flags=None, stream=None, noalloc=False,
                 wall_reflections=False, caustic_uniform=False):
    """E[f, c, n] (complex64 for precision 0, complex128 for 1) and flags[n].

    spheres [ns, 4], cylinders [nc, 5], rx [n, 3]: float32 GPU tensors;
    freqs [nf]: float64 GPU tensor; source: a ``Source`` (``make_source``).
    ``noalloc``: call utd_smooth_field_noalloc (the library's static scratch;
    pass ``out`` and ``flags`` to keep the call free of allocations).
    """
    torch = _torch()
    lib = load_library()
    fn = lib.utd_smooth_field_noalloc if noalloc else lib.utd_smooth_field
    _dev(rx, torch.float32, (3,), "rx")
    _dev(freqs, torch.float64, None, "freqs")
    b, keep = _bodies(spheres, cylinders)
    n, nf = rx.shape[0], freqs.shape[0]
    cdt = torch.complex64 if precision == 0 else torch.complex128
    if out is None:
        out = torch.empty((nf, 3, n), dtype=cdt, device=rx.device)
    if flags is None:
        flags = torch.empty((n,), dtype=torch.uint8, device=rx.device)
    opt = make_options(precision, l_enc, bodies_occlude, lit_branch, caustic_guard, wall_reflections,
                       caustic_uniform)
    _check(fn(scene.handle if scene is not None else None, ctypes.byref(b), ctypes.byref(source),
                                rx.data_ptr() if n else None, n, freqs.data_ptr() if nf else None, nf,
                                ctypes.byref(opt), out.data_ptr() if out.numel() else None,
                                flags.data_ptr() if n else None, _stream(stream)))
    return out, flags


def smooth_field_backward(scene, spheres, cylinders, source, rx, freqs, grad_E, precision=0, l_enc=0,
                          bodies_occlude=True, lit_branch=True, caustic_guard=1e-6, stream=None):
    """Gradients of L with dL/dE = grad_E ([nf, 3, n], complex64 for precision 0,
    complex128 for 1): returns (d_sph [ns, 4], d_cyl [nc, 3], d_tx [3]) on the GPU,
    float32 or float64 by precision.  d_cyl columns are (cx, cy, a)."""
    torch = _torch()
    lib = load_library()
    _dev(rx, torch.float32, (3,), "rx")
    _dev(freqs, torch.float64, None, "freqs")
    b, keep = _bodies(spheres, cylinders)
    n, nf = rx.shape[0], freqs.shape[0]
    cdt = torch.complex64 if precision == 0 else torch.complex128
    rdt = torch.float32 if precision == 0 else torch.float64
    _dev(grad_E, cdt, (3, n), "grad_E")
    if grad_E.shape[0] != nf:
        raise ValueError("grad_E must have shape [n_f, 3, n_rx]")
    d_sph = torch.empty((b.n_sph, 4), dtype=rdt, device=rx.device)
    d_cyl = torch.empty((b.n_cyl, 3), dtype=rdt, device=rx.device)
    d_tx = torch.empty((3,), dtype=rdt, device=rx.device)
    opt = make_options(precision, l_enc, bodies_occlude, lit_branch, caustic_guard)
    _check(lib.utd_smooth_field_backward(
        scene.handle if scene is not None else None, ctypes.byref(b), ctypes.byref(source),
        rx.data_ptr() if n else None, n, freqs.data_ptr() if nf else None, nf, ctypes.byref(opt),
        grad_E.data_ptr() if grad_E.numel() else None, d_cyl.data_ptr() if d_cyl.numel() else None,
        d_sph.data_ptr() if d_sph.numel() else None, d_tx.data_ptr(), _stream(stream)))
    return d_sph, d_cyl, d_tx


class ForwardState:
    """The classification, visibility and path records of one forward call,
    kept on the device for ``smooth_field_backward_saved`` (the library's
    utd_forward_state).  ``release()`` frees it on the given stream; it is
    also released when the object is collected."""

    def __init__(self, handle, n_sph, n_cyl, n_rx, n_f, precision, device, stream):
        self.handle = handle
        self.n_sph, self.n_cyl, self.n_rx, self.n_f = n_sph, n_cyl, n_rx, n_f
        # the stream of the last call that used the state: freeing there
        # orders the release after that call
        self.precision, self.device, self.stream = precision, device, stream

    def release(self, stream=None):
        if self.handle:
            h, self.handle = self.handle, None
            _check(load_library().utd_forward_state_release(h, _stream(stream if stream is not None
                                                                        else self.stream)))

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def smooth_field_saved(scene, spheres, cylinders, source, rx, freqs, precision=0, l_enc=0, bodies_occlude=True,
                       lit_branch=True, caustic_guard=1e-6, out=None, flags=None, stream=None):
    """``smooth_field`` that also returns a ``ForwardState`` for the adjoint:
    (E, flags, state)."""
    torch = _torch()
    lib = load_library()
    _dev(rx, torch.float32, (3,), "rx")
    _dev(freqs, torch.float64, None, "freqs")
    b, keep = _bodies(spheres, cylinders)
    n, nf = rx.shape[0], freqs.shape[0]
    cdt = torch.complex64 if precision == 0 else torch.complex128
    if out is None:
        out = torch.empty((nf, 3, n), dtype=cdt, device=rx.device)
    if flags is None:
        flags = torch.empty((n,), dtype=torch.uint8, device=rx.device)
    opt = make_options(precision, l_enc, bodies_occlude, lit_branch, caustic_guard)
    h = ctypes.c_void_p()
    _check(lib.utd_smooth_field_saved(scene.handle if scene is not None else None, ctypes.byref(b),
                                      ctypes.byref(source), rx.data_ptr() if n else None, n,
                                      freqs.data_ptr() if nf else None, nf, ctypes.byref(opt),
                                      out.data_ptr() if out.numel() else None, flags.data_ptr() if n else None,
                                      ctypes.byref(h), _stream(stream)))
    st = ForwardState(h.value, b.n_sph, b.n_cyl, n, nf, precision, rx.device,
                      stream if stream is not None else torch.cuda.current_stream())
    return out, flags, st


def smooth_field_backward_saved(state, grad_E, stream=None):
    """Gradients from a ``ForwardState``: (d_sph [ns, 4], d_cyl [nc, 3],
    d_tx [3]) exactly as ``smooth_field_backward`` at the forward's inputs."""
    torch = _torch()
    if not state.handle:
        raise ValueError("the forward state was released")
    cdt = torch.complex64 if state.precision == 0 else torch.complex128
    rdt = torch.float32 if state.precision == 0 else torch.float64
    _dev(grad_E, cdt, (3, state.n_rx), "grad_E")
    if grad_E.shape[0] != state.n_f:
        raise ValueError("grad_E must have shape [n_f, 3, n_rx]")
    d_sph = torch.empty((state.n_sph, 4), dtype=rdt, device=state.device)
    d_cyl = torch.empty((state.n_cyl, 3), dtype=rdt, device=state.device)
    d_tx = torch.empty((3,), dtype=rdt, device=state.device)
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(load_library().utd_smooth_field_backward_saved(
        state.handle, grad_E.data_ptr() if grad_E.numel() else None, d_cyl.data_ptr() if d_cyl.numel() else None,
        d_sph.data_ptr() if d_sph.numel() else None, d_tx.data_ptr(), _stream(s)))
    state.stream = s
    return d_sph, d_cyl, d_tx


def _autograd_function():
    torch = _torch()

    class _SmoothField(torch.autograd.Function):
        @staticmethod
        def forward(ctx, spheres, cylinders, tx_pos, rx, freqs, scene, dipole, amplitude, kw):
            src = make_source([float(v) for v in tx_pos.detach().cpu().tolist()], dipole, amplitude)
            sph, cyl = spheres.detach().contiguous(), cylinders.detach().contiguous()
            # the forward keeps its classification and records for the backward
            E, _, st = smooth_field_saved(scene, sph, cyl, src, rx, freqs, **kw)
            ctx.save_for_backward(sph, cyl)
            ctx.state, ctx.tx_meta = st, (tx_pos.dtype, tx_pos.device)
            return E

        @staticmethod
        def backward(ctx, gE):
            sph, cyl = ctx.saved_tensors
            d_sph, d_cyl3, d_tx = smooth_field_backward_saved(ctx.state,
                                                              gE.resolve_conj().resolve_neg().contiguous())
            d_cyl = torch.zeros(cyl.shape, dtype=d_cyl3.dtype, device=cyl.device)
            d_cyl[:, 0:2] = d_cyl3[:, 0:2]
            d_cyl[:, 4] = d_cyl3[:, 2]
            dt, dev = ctx.tx_meta
            return (d_sph.to(sph.dtype), d_cyl.to(cyl.dtype), d_tx.to(dtype=dt, device=dev),
                    None, None, None, None, None, None)

    return _SmoothField


def field(scene, spheres, cylinders, tx_pos, rx, freqs, dipole=(0.0, 0.0, 1.0), amplitude=1.0, precision=0,
          l_enc=0, bodies_occlude=True, lit_branch=True, caustic_guard=1e-6):
    """Differentiable forward field: E[f, c, n] as ``smooth_field``, with
    PyTorch autograd through ``utd_smooth_field_backward`` for ``spheres``,
    ``cylinders`` (columns cx, cy, a; heights get zero) and ``tx_pos`` (a
    3-vector tensor, CPU or GPU)."""
    kw = dict(precision=precision, l_enc=l_enc, bodies_occlude=bodies_occlude, lit_branch=lit_branch,
              caustic_guard=caustic_guard)
    return _autograd_function().apply(spheres, cylinders, tx_pos, rx, freqs, scene, dipole, amplitude, kw)


def batched_config(tile_rx, blocks_per_cu):
    """Tile shape of the batched kernel (receivers per work item, workgroups per CU)."""
    _check(load_library().utd_batched_config(int(tile_rx), int(blocks_per_cu)))


def smooth_field_batched(scene, body_off, cylinders, rx_off, rx, source, freqs, precision=0, l_enc=0,
                         bodies_occlude=True, lit_branch=True, caustic_guard=1e-6, out=None, flags=None, stream=None,
                         caustic_uniform=False):
    """Fields of many frames in one call.  body_off, rx_off: int64 GPU tensors
    [n_frames + 1]; cylinders [n_cyl, 5], rx [n_rx, 3]: float32 GPU tensors.
    Returns (E, flags): E is a flat complex tensor of 3 * n_f * n_rx elements,
    frame f's [n_f, 3, n_rx_f] block starting at 3 * n_f * rx_off[f]."""
    torch = _torch()
    lib = load_library()
    _dev(rx, torch.float32, (3,), "rx")
    _dev(cylinders, torch.float32, (5,), "cylinders")
    _dev(freqs, torch.float64, None, "freqs")
    _dev(body_off, torch.int64, None, "body_off")
    _dev(rx_off, torch.int64, None, "rx_off")
    if body_off.dim() != 1 or rx_off.shape != body_off.shape:
        raise ValueError("body_off and rx_off must be 1-D of equal length n_frames + 1")
    n_frames = body_off.shape[0] - 1
    n, nf, nc = rx.shape[0], freqs.shape[0], cylinders.shape[0]
    cdt = torch.complex64 if precision == 0 else torch.complex128
    if out is None:
        out = torch.empty((3 * nf * n,), dtype=cdt, device=rx.device)
    if flags is None:
        flags = torch.empty((n,), dtype=torch.uint8, device=rx.device)
    opt = make_options(precision, l_enc, bodies_occlude, lit_branch, caustic_guard,
                       caustic_uniform=caustic_uniform)
    _check(lib.utd_smooth_field_batched(
        scene.handle if scene is not None else None, max(n_frames, 0), body_off.data_ptr(),
        cylinders.data_ptr() if nc else None, nc, rx_off.data_ptr(), rx.data_ptr() if n else None, n,
        ctypes.byref(source), freqs.data_ptr() if nf else None, nf, ctypes.byref(opt),
        out.data_ptr() if out.numel() else None, flags.data_ptr() if n else None, _stream(stream)))
    return out, flags


def profile_enable(on=True):
    """Record HIP event pairs around every kernel launch (measurement only)."""
    load_library().utd_profile_enable(int(bool(on)))


def profile_read():
    """{kernel: (total_ms, launches)} since the last read; waits for the events."""
    lib = load_library()
    ms = (ctypes.c_double * len(KERNELS))()
    cnt = (ctypes.c_int64 * len(KERNELS))()
    _check(lib.utd_profile_read(ctypes.cast(ms, ctypes.c_void_p), ctypes.cast(cnt, ctypes.c_void_p)))
    return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNELS)}


def path_census(scene, spheres, cylinders, source, rx, l_enc=0, bodies_occlude=True, lit_branch=True,
                caustic_guard=1e-6, stream=None):
    """Counts of evaluated paths: dict with creeping (per side/ell), reflections,
    caustic drops, line-of-sight receivers and receivers inside bodies."""
    torch = _torch()
    lib = load_library()
    _dev(rx, torch.float32, (3,), "rx")
    b, keep = _bodies(spheres, cylinders)
    opt = make_options(0, l_enc, bodies_occlude, lit_branch, caustic_guard)
    counts = (ctypes.c_int64 * 10)()
    _check(lib.utd_path_census(scene.handle if scene is not None else None, ctypes.byref(b), ctypes.byref(source),
                               rx.data_ptr() if rx.shape[0] else None, rx.shape[0], ctypes.byref(opt),
                               ctypes.cast(counts, ctypes.c_void_p), _stream(stream)))
    c = list(counts)
    return dict(creeping=sum(c[:6]), creeping_by_bit=c[:6], reflections=c[6], caustic=c[7], los=c[8], inside=c[9],
                paths=sum(c[:7]))


def path_masks(scene, spheres, cylinders, source, rx, precision=0, l_enc=0, bodies_occlude=True, lit_branch=True,
               caustic_guard=1e-6, stream=None):
    """Visibility decisions of ``smooth_field`` for the same inputs:
    (mask [n_bodies, n_rx] uint8, flags [n_rx] uint8) on the GPU; bodies are
    ordered spheres first, then cylinders.  Mask bits: 2 ell + side for the
    creeping paths, 6 the reflection, 7 a caustic drop."""
    torch = _torch()
    lib = load_library()
    _dev(rx, torch.float32, (3,), "rx")
    b, keep = _bodies(spheres, cylinders)
    n = rx.shape[0]
    nb = b.n_sph + b.n_cyl
    mask = torch.empty((nb, n), dtype=torch.uint8, device=rx.device)
    flags = torch.empty((n,), dtype=torch.uint8, device=rx.device)
    opt = make_options(precision, l_enc, bodies_occlude, lit_branch, caustic_guard)
    _check(lib.utd_path_masks(scene.handle if scene is not None else None, ctypes.byref(b), ctypes.byref(source),
                              rx.data_ptr() if n else None, n, ctypes.byref(opt),
                              mask.data_ptr() if mask.numel() else None, flags.data_ptr() if n else None,
                              _stream(stream)))
    return mask, flags


def input_status():
    """Waits for the device; returns and clears the BAD_* bits raised since the last read."""
    v = ctypes.c_uint32(0)
    _check(load_library().utd_input_status(ctypes.cast(ctypes.pointer(v), ctypes.c_void_p)))
    return int(v.value)


def wall_masks(scene, spheres, cylinders, source, rx, precision=0, l_enc=0, bodies_occlude=True, lit_branch=True,
               caustic_guard=1e-6, stream=None):
    """Wall-bounce decisions of ``smooth_field(..., wall_reflections=True)``:
    uint64 words [n_rx, n_planes] as a GPU int64 tensor (bit 0 the wall's
    own ray; body b bits 1 + 6 b + k, k = 0/1 wall then creeping side +/-, 2
    wall then reflection, 3/4 creeping then wall, 5 reflection then wall)."""
    torch = _torch()
    lib = load_library()
    _dev(rx, torch.float32, (3,), "rx")
    b, keep = _bodies(spheres, cylinders)
    n = rx.shape[0]
    n_planes = int(lib.utd_scene_planes(scene.handle, None)) if scene is not None else 0
    out = torch.zeros((n, n_planes), dtype=torch.int64, device=rx.device)
    opt = make_options(precision, l_enc, bodies_occlude, lit_branch, caustic_guard, True)
    _check(lib.utd_wall_masks(scene.handle if scene is not None else None, ctypes.byref(b), ctypes.byref(source),
                              rx.data_ptr() if n else None, n, ctypes.byref(opt),
                              out.data_ptr() if out.numel() else None, _stream(stream)))
    return out
