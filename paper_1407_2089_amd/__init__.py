"""Python binding of libvr, the MI355X stereo multichannel volume ray caster.

The functions named ``vr_*`` mirror the C ABI in ``include/vr.h`` one to one
and only marshal arguments through ctypes: every step of rendering runs in
the library's HIP kernels.  A non-OK status raises :class:`VrError`.  The
small classes at the bottom (``Context``, ``Volume``) use PyTorch for device
memory and streams and call the same functions.

The library must be built (``__graft_entry__.build()``); importing this
module never falls back to another implementation.
"""
from __future__ import annotations

import ctypes as C
import os

__all__ = [
    "VrError", "lib", "vr_init", "vr_shutdown", "vr_volume_storage_bytes",
    "vr_create_volume", "vr_upload_frame", "vr_destroy_volume", "vr_set_transfer",
    "vr_render", "vr_render_batch", "vr_submit", "vr_poll", "vr_release",
    "vr_last_error", "vr_debug_sample", "Context", "Volume", "VR_U8", "VR_U16",
    "VR_FP32", "VR_FP16", "VR_ORTHO", "VR_PERSPECTIVE", "vr_denoise_workspace_bytes",
    "vr_remove_background", "vr_mrf_denoise", "gaussian_weights", "remove_background",
    "mrf_denoise", "vr_stream_frame", "vr_stream_ready", "vr_gaussian_weights",
    "vr_tune_batch", "vr_render_batch_noalloc", "vr_tune_layout",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvr.so")

VR_OK, VR_ERR_INVALID_ARG, VR_ERR_OUT_OF_MEMORY, VR_ERR_NOT_FOUND = 0, -1, -2, -3
VR_ERR_BUSY, VR_ERR_DEVICE, VR_ERR_UNSUPPORTED = -4, -5, -6
VR_U8, VR_U16 = 1, 2
VR_FP32, VR_FP16 = 0, 1
VR_ORTHO, VR_PERSPECTIVE = 0, 1
STATUS_NAMES = {0: "VR_OK", -1: "VR_ERR_INVALID_ARG", -2: "VR_ERR_OUT_OF_MEMORY",
                -3: "VR_ERR_NOT_FOUND", -4: "VR_ERR_BUSY", -5: "VR_ERR_DEVICE",
                -6: "VR_ERR_UNSUPPORTED"}


class VrError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")


class vr_volume_desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("channels", C.c_int32), ("frames", C.c_int32), ("dtype", C.c_int32),
                ("bits", C.c_int32), ("spacing", C.c_float * 3), ("origin", C.c_float * 3),
                ("brick", C.c_int32 * 3), ("row_pairs", C.c_int32)]


class vr_transfer(C.Structure):
    _fields_ = [("lo", C.c_float), ("hi", C.c_float), ("curve", C.c_float),
                ("alpha_mul", C.c_float), ("rgb", C.c_float * 3), ("visible", C.c_int32)]


class vr_camera(C.Structure):
    _fields_ = [("projection", C.c_int32), ("center", C.c_float * 3),
                ("forward", C.c_float * 3), ("up", C.c_float * 3), ("fov_y", C.c_float),
                ("ortho_height", C.c_float), ("eye_separation", C.c_float),
                ("convergence", C.c_float)]


class vr_light(C.Structure):
    _fields_ = [("enabled", C.c_int32), ("direction", C.c_float * 3), ("ambient", C.c_float),
                ("diffuse", C.c_float)]


class vr_render_req(C.Structure):
    _fields_ = [("vol", C.c_void_p), ("frame", C.c_int32), ("cam", vr_camera),
                ("width", C.c_int32), ("height", C.c_int32), ("stereo", C.c_int32),
                ("step", C.c_float), ("term_alpha", C.c_float),
                ("background", C.c_float * 4), ("precision", C.c_int32),
                ("out_rgba", C.c_void_p), ("out_samples", C.c_void_p),
                ("light", vr_light)]


class vr_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("dtype", C.c_int32),
                ("bits", C.c_int32)]


class vr_lowpass(C.Structure):
    _fields_ = [("w", C.POINTER(C.c_uint32) * 3), ("taps", C.c_int32 * 3), ("shift", C.c_int32)]


class vr_mrf_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("delta", C.c_int32), ("sigma", C.c_double),
                ("rms", C.c_double)]


class vr_ticket_info(C.Structure):
    _fields_ = [("state", C.c_int32), ("err", C.c_int32), ("t_arrive_ns", C.c_uint64),
                ("t_admit_ns", C.c_uint64), ("t_start_ns", C.c_uint64),
                ("t_done_ns", C.c_uint64), ("samples", C.c_uint64), ("rays", C.c_uint64)]


_lib = None


def lib():
    """The loaded libvr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        # PyTorch links its own HIP runtime under the unversioned name, so a
        # library loaded before it would bring a second runtime into the
        # process, and the second one to start finds no device.  Importing
        # torch first makes libvr bind to the runtime torch already holds.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        P, S = C.c_void_p, C.c_int
        sig = {
            "vr_init": [C.c_int32, C.c_uint64, C.POINTER(C.c_void_p)],
            "vr_shutdown": [P],
            "vr_volume_storage_bytes": [C.POINTER(vr_volume_desc), C.POINTER(C.c_uint64)],
            "vr_create_volume": [P, C.POINTER(vr_volume_desc), P, C.c_uint64,
                                 C.POINTER(C.c_void_p)],
            "vr_upload_frame": [P, C.c_int32, P, P],
            "vr_stream_frame": [P, C.c_int32, P, P, C.c_uint64, P, P],
            "vr_stream_ready": [P, C.c_int32, P],
            "vr_destroy_volume": [P],
            "vr_set_transfer": [P, C.c_int32, C.POINTER(vr_transfer)],
            "vr_render": [P, C.POINTER(vr_render_req), P],
            "vr_render_batch": [P, C.POINTER(vr_render_req), C.c_int32, P],
            "vr_render_batch_noalloc": [P, C.POINTER(vr_render_req), C.c_int32, P],
            "vr_tune_batch": [P, C.POINTER(vr_render_req), C.c_int32, P,
                              C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
            "vr_tune_layout": [P, C.POINTER(vr_volume_desc), C.POINTER(vr_transfer), P,
                               C.POINTER(vr_render_req), C.c_int32, C.c_int32, C.c_uint64, P,
                               C.POINTER(C.c_float)],
            "vr_submit": [P, C.POINTER(vr_render_req), C.POINTER(C.c_uint64)],
            "vr_poll": [P, C.c_uint64, C.POINTER(vr_ticket_info)],
            "vr_release": [P, C.c_uint64],
            "vr_debug_sample": [P, C.c_int32, P, C.c_int32, P, P],
            "vr_denoise_workspace_bytes": [C.POINTER(vr_grid), C.POINTER(C.c_uint64)],
            "vr_gaussian_weights": [C.c_double, C.c_int32, C.c_int32, P, C.c_int32,
                                    C.POINTER(C.c_int32)],
            "vr_remove_background": [P, C.POINTER(vr_grid), C.POINTER(vr_lowpass), P, P, P, P,
                                     C.c_uint64, P],
            "vr_mrf_denoise": [P, C.POINTER(vr_grid), C.c_int32, P, P, P, C.c_uint64, P,
                               C.POINTER(vr_mrf_info)],
            "vr_test_fake_backend": [P, C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                     C.c_double],
            "vr_test_batch_tile": [P, C.c_int32, C.c_int32],
            "vr_test_plain_tile": [P, C.c_int32, C.c_int32],
            "vr_test_block_map": [C.c_int32, C.c_void_p],
            "vr_test_clear_skip": [P, C.c_int32],
            "vr_test_large_addressing": [P, C.c_int32],
            "vr_test_volume_large": [P, C.POINTER(C.c_int32)],
            "vr_test_cell_shift": [P, C.c_int32],
            "vr_test_transparent_max": [C.c_float, C.c_float, C.c_int32, C.POINTER(C.c_float),
                                        C.POINTER(C.c_float), C.POINTER(C.c_int32)],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = S
        L.vr_last_error.argtypes = []
        L.vr_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def vr_last_error() -> str:
    return lib().vr_last_error().decode()


def _check(status):
    if status != VR_OK:
        raise VrError(status, vr_last_error())
    return status


def _ptr(x):
    """Device address of a torch tensor, an int, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


# ------------------------------------------------------------- C ABI mirror

def vr_init(device: int = 0, mem_budget_bytes: int = 0):
    out = C.c_void_p()
    _check(lib().vr_init(device, mem_budget_bytes, C.byref(out)))
    return out.value


def vr_shutdown(ctx):
    _check(lib().vr_shutdown(ctx))


def vr_volume_storage_bytes(desc: vr_volume_desc) -> int:
    out = C.c_uint64()
    _check(lib().vr_volume_storage_bytes(C.byref(desc), C.byref(out)))
    return out.value


def vr_create_volume(ctx, desc: vr_volume_desc, dev_storage, storage_bytes: int):
    out = C.c_void_p()
    _check(lib().vr_create_volume(ctx, C.byref(desc), _ptr(dev_storage), storage_bytes,
                                  C.byref(out)))
    return out.value


def vr_upload_frame(vol, frame: int, dev_src, stream=None):
    _check(lib().vr_upload_frame(vol, frame, _ptr(dev_src), _stream(stream)))


def vr_destroy_volume(vol):
    _check(lib().vr_destroy_volume(vol))


def vr_set_transfer(vol, channel: int, tf: vr_transfer):
    _check(lib().vr_set_transfer(vol, channel, C.byref(tf)))


def vr_render(ctx, req: vr_render_req, stream=None):
    _check(lib().vr_render(ctx, C.byref(req), _stream(stream)))


def vr_render_batch(ctx, reqs, stream=None):
    n = len(reqs)
    arr = (vr_render_req * max(n, 1))(*reqs)
    _check(lib().vr_render_batch(ctx, arr, n, _stream(stream)))


def vr_render_batch_noalloc(ctx, reqs, stream=None):
    n = len(reqs)
    arr = (vr_render_req * max(n, 1))(*reqs)
    _check(lib().vr_render_batch_noalloc(ctx, arr, n, _stream(stream)))


def vr_tune_batch(ctx, reqs, stream=None):
    """Autotune the batched launch for this batch's shape class; returns the
    chosen (wave_w, wave_h)."""
    n = len(reqs)
    arr = (vr_render_req * max(n, 1))(*reqs)
    w, h = C.c_int32(), C.c_int32()
    _check(lib().vr_tune_batch(ctx, arr, n, _stream(stream), C.byref(w), C.byref(h)))
    return w.value, h.value


def vr_tune_layout(ctx, desc: vr_volume_desc, tfs, dev_frame, views, reps=10, max_bytes=0,
                   stream=None):
    """Choose the layout of `desc` by timing `views` on each candidate built
    from dev_frame; updates desc.brick and desc.row_pairs in place and
    returns the winner's summed median time in ms."""
    tf_arr = (vr_transfer * len(tfs))(*[t if isinstance(t, vr_transfer) else
                                        make_transfer(t.lo, t.hi, t.curve, t.alpha_mul, t.rgb,
                                                      t.visible) for t in tfs])
    arr = (vr_render_req * max(len(views), 1))(*views)
    ms = C.c_float()
    _check(lib().vr_tune_layout(ctx, C.byref(desc), tf_arr, _ptr(dev_frame), arr, len(views),
                                reps, max_bytes, _stream(stream), C.byref(ms)))
    return ms.value


def vr_submit(ctx, req: vr_render_req) -> int:
    t = C.c_uint64()
    _check(lib().vr_submit(ctx, C.byref(req), C.byref(t)))
    return t.value


def vr_poll(ctx, ticket: int) -> vr_ticket_info:
    info = vr_ticket_info()
    _check(lib().vr_poll(ctx, ticket, C.byref(info)))
    return info


def vr_release(ctx, ticket: int):
    _check(lib().vr_release(ctx, ticket))


def vr_debug_sample(vol, frame: int, pts, n: int, out, stream=None):
    _check(lib().vr_debug_sample(vol, frame, _ptr(pts), n, _ptr(out), _stream(stream)))


# ------------------------------------------------------------- denoising

def make_grid(nx, ny, nz, dtype, bits):
    return vr_grid(nx, ny, nz, dtype, bits)


def vr_denoise_workspace_bytes(grid) -> int:
    n = C.c_uint64()
    _check(lib().vr_denoise_workspace_bytes(C.byref(grid), C.byref(n)))
    return n.value


def make_lowpass(wx, wy, wz, shift):
    """vr_lowpass from three integer weight lists (kept alive on the struct)."""
    arrs = [(C.c_uint32 * len(w))(*[int(v) for v in w]) for w in (wx, wy, wz)]
    lp = vr_lowpass((C.POINTER(C.c_uint32) * 3)(*[C.cast(a, C.POINTER(C.c_uint32))
                                                    for a in arrs]),
                    (C.c_int32 * 3)(*[len(w) for w in (wx, wy, wz)]), int(shift))
    lp._keep = arrs
    return lp


def vr_remove_background(ctx, grid, lp, src, dst, background, workspace, workspace_bytes,
                         stream=None):
    _check(lib().vr_remove_background(ctx, C.byref(grid), C.byref(lp), _ptr(src), _ptr(dst),
                                      _ptr(background), _ptr(workspace), workspace_bytes,
                                      _stream(stream)))


def vr_mrf_denoise(ctx, grid, max_iters, src, dst, workspace, workspace_bytes, stream=None):
    info = vr_mrf_info()
    _check(lib().vr_mrf_denoise(ctx, C.byref(grid), max_iters, _ptr(src), _ptr(dst),
                                _ptr(workspace), workspace_bytes, _stream(stream),
                                C.byref(info)))
    return info


def vr_gaussian_weights(sigma: float, shift: int = 14, radius: int = -1):
    """Quantised Gaussian low-pass weights from the library (a list of ints
    summing to 2^shift; radius -1: min(64, ceil(3 sigma)))."""
    buf = (C.c_uint32 * 129)()
    taps = C.c_int32()
    _check(lib().vr_gaussian_weights(float(sigma), int(shift), int(radius), buf, 129,
                                     C.byref(taps)))
    return [int(buf[i]) for i in range(taps.value)]


def gaussian_weights(sigma, shift=14, radius=None):
    """vr_gaussian_weights with radius None meaning the library default."""
    return vr_gaussian_weights(sigma, shift, -1 if radius is None else radius)


def _grid_of(vol, bits):
    import torch
    nz, ny, nx = vol.shape
    dtype = VR_U8 if vol.dtype == torch.uint8 else VR_U16
    return make_grid(nx, ny, nz, dtype, bits)


def _workspace(grid, device):
    import torch
    n = vr_denoise_workspace_bytes(grid)
    return torch.empty(n, dtype=torch.uint8, device=device), n


def remove_background(ctx, vol, wx, wy, wz, shift, bits, stream=None):
    """Background removal of a [Z][Y][X] uint8 / int16-viewed uint16 device
    tensor: returns (denoised, background) as new tensors of the same type."""
    import torch
    grid = _grid_of(vol, bits)
    ws, n = _workspace(grid, vol.device)
    dst, bg = torch.empty_like(vol), torch.empty_like(vol)
    vr_remove_background(ctx.ptr, grid, make_lowpass(wx, wy, wz, shift), vol, dst, bg, ws, n,
                         stream)
    return dst, bg


def mrf_denoise(ctx, vol, bits, max_iters, stream=None):
    """Sign-diffusion denoising of a [Z][Y][X] device tensor: (result, info)."""
    import torch
    grid = _grid_of(vol, bits)
    ws, n = _workspace(grid, vol.device)
    dst = torch.empty_like(vol)
    info = vr_mrf_denoise(ctx.ptr, grid, max_iters, vol, dst, ws, n, stream)
    return dst, info


def vr_stream_frame(vol, slot: int, host_src, dev_staging, staging_bytes: int, copy_stream,
                    render_stream):
    """host_src: a (pinned) CPU tensor or an integer address."""
    src = host_src if isinstance(host_src, int) else host_src.data_ptr()
    _check(lib().vr_stream_frame(vol, slot, src, _ptr(dev_staging), staging_bytes,
                                 _stream(copy_stream), _stream(render_stream)))


def vr_stream_ready(vol, slot: int, render_stream):
    _check(lib().vr_stream_ready(vol, slot, _stream(render_stream)))


def vr_test_batch_tile(ctx, wave_w=0, wave_h=0):
    _check(lib().vr_test_batch_tile(ctx, wave_w, wave_h))


def vr_test_plain_tile(ctx, wave_w=0, wave_h=0):
    _check(lib().vr_test_plain_tile(ctx, wave_w, wave_h))


def vr_test_clear_skip(ctx, on):
    """on: False/0 no skipping, True/1 both skips (default), 2 the per-sample
    test only (every sample walked)."""
    _check(lib().vr_test_clear_skip(ctx, int(on)))


def vr_test_large_addressing(ctx, on: bool):
    _check(lib().vr_test_large_addressing(ctx, int(bool(on))))


def vr_test_cell_shift(ctx, shift: int = 3):
    _check(lib().vr_test_cell_shift(ctx, int(shift)))


def vr_test_volume_large(vol) -> bool:
    out = C.c_int32()
    _check(lib().vr_test_volume_large(vol, C.byref(out)))
    return bool(out.value)


def vr_test_transparent_max(lo: float, hi: float, bits: int):
    """(scale, bias, tmax) of the transparent-sample test (host-only)."""
    scale, bias, tmax = C.c_float(), C.c_float(), C.c_int32()
    _check(lib().vr_test_transparent_max(lo, hi, bits, C.byref(scale), C.byref(bias),
                                         C.byref(tmax)))
    return scale.value, bias.value, tmax.value


def vr_test_block_map(nblocks: int):
    """Tile rendered by each hardware block of a plain launch (host-only)."""
    import numpy as np
    out = np.zeros(max(nblocks, 1), np.int32)
    _check(lib().vr_test_block_map(nblocks, out.ctypes.data))
    return out[:nblocks]


def vr_test_fake_backend(ctx, slots: int, ns_per_ray: float, fail_width: int = -1,
                         max_batch: int = 32, launch_ms: float = 0.0):
    _check(lib().vr_test_fake_backend(ctx, slots, ns_per_ray, fail_width, max_batch,
                                      float(launch_ms)))


# ---------------------------------------------------------- record helpers

def make_transfer(lo=0.0, hi=1.0, curve=0.0, alpha_mul=1.0, rgb=(1.0, 1.0, 1.0), visible=True):
    return vr_transfer(lo, hi, curve, alpha_mul, (C.c_float * 3)(*rgb), int(bool(visible)))


def make_camera(cam) -> vr_camera:
    """vr_camera from any object with the synth.Cam fields."""
    f3 = C.c_float * 3
    proj = VR_PERSPECTIVE if cam.projection in ("perspective", VR_PERSPECTIVE) else VR_ORTHO
    return vr_camera(proj, f3(*cam.center), f3(*cam.forward), f3(*cam.up), cam.fov_y,
                     cam.ortho_height, cam.eye_separation, cam.convergence)


def make_light(light):
    """vr_light from an object with direction, ambient and diffuse (None: off)."""
    if light is None:
        return vr_light()
    return vr_light(1, (C.c_float * 3)(*light.direction), light.ambient, light.diffuse)


def make_request(vol, frame, cam, width, height, stereo, step, term_alpha, out_rgba,
                 background=(0.0, 0.0, 0.0, 0.0), precision=VR_FP32, out_samples=None,
                 light=None):
    return vr_render_req(vol, frame, make_camera(cam), width, height, int(bool(stereo)),
                         step, term_alpha, (C.c_float * 4)(*background), precision,
                         _ptr(out_rgba), _ptr(out_samples), make_light(light))


# --------------------------------------------------------- torch helpers

class Context:
    """A libvr context on one GPU (torch provides memory and streams)."""

    def __init__(self, device: int = 0, mem_budget_bytes: int = 0):
        self.device = device
        self.ptr = vr_init(device, mem_budget_bytes)

    def close(self):
        if self.ptr:
            vr_shutdown(self.ptr)
            self.ptr = None


class Volume:
    """A resident series in torch-allocated device storage."""

    def __init__(self, ctx: Context, dims, channels, frames=1, dtype=VR_U8, bits=None,
                 spacing=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0), brick=(0, 0, 0),
                 row_pairs=False, storage_bytes=None):
        import torch
        nx, ny, nz = dims
        bits = bits if bits is not None else (8 if dtype == VR_U8 else 16)
        self.desc = vr_volume_desc(nx, ny, nz, channels, frames, dtype, bits,
                                   (C.c_float * 3)(*spacing), (C.c_float * 3)(*origin),
                                   (C.c_int32 * 3)(*brick), int(bool(row_pairs)))
        self.bytes = storage_bytes or vr_volume_storage_bytes(self.desc)
        self.storage = torch.empty(self.bytes + 256, dtype=torch.uint8,
                                   device=f"cuda:{ctx.device}")
        base = self.storage.data_ptr()
        self.base = (base + 255) & ~255
        self.ctx = ctx
        self.ptr = vr_create_volume(ctx.ptr, self.desc, self.base, self.bytes)
        self.channels = channels

    def upload(self, frame, src, stream=None):
        """src: torch device tensor [C][Z][Y][X] of uint8 / int16-viewed uint16."""
        if not src.is_contiguous():
            raise ValueError("source frame must be contiguous")
        vr_upload_frame(self.ptr, frame, src, stream)

    def set_transfer(self, channel, tf):
        if not isinstance(tf, vr_transfer):
            tf = make_transfer(tf.lo, tf.hi, tf.curve, tf.alpha_mul, tf.rgb, tf.visible)
        vr_set_transfer(self.ptr, channel, tf)

    def destroy(self):
        if self.ptr:
            vr_destroy_volume(self.ptr)
            self.ptr = None
