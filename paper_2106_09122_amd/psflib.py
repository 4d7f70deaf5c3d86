"""Python binding of the psflib C ABI (``include/psflib.h``).

Argument marshalling only: every step of the operator runs in the HIP
kernels of ``libpsflib.so``.  PyTorch supplies device memory (tensors) and
the current HIP stream.  If the shared library is missing this module raises
at import time; there is no fallback implementation.

Low-level functions keep the C names without the ``psflib_`` prefix
(``build``, ``apply``, ``apply_adjoint``, ``apply_batched``, ...) and take
device pointers as integers.  :class:`Library` wraps them for torch tensors.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG_DIR, "libpsflib.so")

OK, ERR_INVALID_ARG, ERR_RADII, ERR_SIZE, ERR_UNSUPPORTED, ERR_DEVICE = range(6)
INTERP = {"linear": 0, "nearest": 1}
OOB = {"clamp": 0, "zero": 1}
STORAGE = {"fp32": 0, "bf16": 1, "fp16": 2}
ROTATE = {"bilinear": 0, "cubic": 1}
FLUX = {"none": 0, "preserve": 1}


class PsflibError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {_status_name(status)}: {message}")


class Desc(ctypes.Structure):
    """Mirror of ``psflib_desc``."""
    _fields_ = [
        ("n", ctypes.c_int32),
        ("n_psf", ctypes.c_int32),
        ("N", ctypes.c_int32),
        ("interp", ctypes.c_int32),
        ("scene_pixscale", ctypes.c_double),
        ("oob", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("rotate", ctypes.c_int32),
        ("flux", ctypes.c_int32),
    ]


def _load():
    # The library must run on the same HIP runtime instance as torch (whose
    # streams and device pointers it receives).  Importing torch first loads
    # torch's libamdhip64; the dynamic linker then resolves this library's
    # libamdhip64.so.7 dependency to that already-loaded copy by its soname.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950) first")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    DP = ctypes.POINTER(Desc)
    sig = {
        "psflib_status_string": (ctypes.c_char_p, [I32]),
        "psflib_last_error": (ctypes.c_char_p, []),
        "psflib_library_bytes": (I32, [DP, ctypes.POINTER(SZ)]),
        "psflib_build": (I32, [DP, P, ctypes.POINTER(ctypes.c_double), P, SZ, P,
                               ctypes.POINTER(P)]),
        "psflib_apply": (I32, [P, P, P, P]),
        "psflib_apply_noalloc": (I32, [P, P, P, P]),
        "psflib_apply_adjoint": (I32, [P, P, P, P]),
        "psflib_apply_batched": (I32, [P, P, P, I32, P]),
        "psflib_column_sums": (I32, [P, P, P]),
        "psflib_get_columns": (I32, [P, P, I32, P, P]),
        "psflib_get_exponents": (I32, [P, P, P]),
        "psflib_get_geometry": (I32, [P, P, P, P]),
        "psflib_render_disk": (I32, [I32, ctypes.c_double, ctypes.c_double, P, P, P]),
        "psflib_grouped_create": (I32, [P, I32, P, P, P, I32, I32, P, ctypes.POINTER(P)]),
        "psflib_grouped_run": (I32, [P, P]),
        "psflib_grouped_chunk": (I32, [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_float)]),
        "psflib_grouped_shape": (I32, [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_float)]),
        "psflib_grouped_set_shape": (I32, [P, ctypes.c_int64, ctypes.c_int32, P]),
        "psflib_grouped_destroy": (None, [P]),
        "psflib_render_disk_grad": (I32, [I32, ctypes.c_double, ctypes.c_double, P, P, P, P]),
        "psflib_chi2": (I32, [ctypes.c_int64, ctypes.c_double, P, P, P, P, P, P]),
        "psflib_destroy": (None, [P]),
        "psflib_probe_hbm_read": (I32, [P, SZ, I32, I32, I32, P, P]),
        "psflib_probe_mfma": (I32, [I32, I32, I32, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()

#: every symbol the header declares
SYMBOLS = (
    "psflib_status_string", "psflib_last_error", "psflib_library_bytes", "psflib_build",
    "psflib_apply", "psflib_apply_noalloc", "psflib_apply_adjoint", "psflib_apply_batched", "psflib_column_sums",
    "psflib_get_columns", "psflib_get_exponents", "psflib_get_geometry", "psflib_destroy",
    "psflib_render_disk", "psflib_render_disk_grad", "psflib_chi2", "psflib_grouped_create",
    "psflib_grouped_run", "psflib_grouped_chunk", "psflib_grouped_shape", "psflib_grouped_set_shape",
    "psflib_grouped_destroy",
    "psflib_probe_hbm_read", "psflib_probe_mfma",
)


def _status_name(s: int) -> str:
    return _lib.psflib_status_string(int(s)).decode()


def _check(status: int, where: str):
    if status != OK:
        raise PsflibError(status, where, _lib.psflib_last_error().decode())


def make_desc(n: int, n_psf: int, N: int, scene_pixscale: float, interp="linear", oob="clamp",
              storage="fp32", rotate="bilinear", flux="none") -> Desc:
    d = Desc()
    d.n, d.n_psf, d.N = int(n), int(n_psf), int(N)
    d.scene_pixscale = float(scene_pixscale)
    d.interp = INTERP[interp] if isinstance(interp, str) else int(interp)
    d.oob = OOB[oob] if isinstance(oob, str) else int(oob)
    d.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    d.rotate = ROTATE[rotate] if isinstance(rotate, str) else int(rotate)
    d.flux = FLUX[flux] if isinstance(flux, str) else int(flux)
    return d


# ---------------------------------------------------------- raw C calls ----
def library_bytes(desc: Desc) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.psflib_library_bytes(ctypes.byref(desc), ctypes.byref(out)), "psflib_library_bytes")
    return int(out.value)


def build(desc: Desc, d_cube: int, radii, d_lib: int, lib_bytes: int, stream: int) -> int:
    r = np.ascontiguousarray(np.asarray(radii, dtype=np.float64))
    h = ctypes.c_void_p()
    _check(_lib.psflib_build(ctypes.byref(desc), ctypes.c_void_p(d_cube),
                             r.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             ctypes.c_void_p(d_lib), ctypes.c_size_t(lib_bytes),
                             ctypes.c_void_p(stream), ctypes.byref(h)), "psflib_build")
    return int(h.value)


def apply(h: int, d_scene: int, d_image: int, stream: int):
    _check(_lib.psflib_apply(ctypes.c_void_p(h), ctypes.c_void_p(d_scene), ctypes.c_void_p(d_image),
                             ctypes.c_void_p(stream)), "psflib_apply")


def apply_noalloc(h: int, d_scene: int, d_image: int, stream: int):
    _check(_lib.psflib_apply_noalloc(ctypes.c_void_p(h), ctypes.c_void_p(d_scene),
                                     ctypes.c_void_p(d_image), ctypes.c_void_p(stream)),
           "psflib_apply_noalloc")


def apply_adjoint(h: int, d_g: int, d_out: int, stream: int):
    _check(_lib.psflib_apply_adjoint(ctypes.c_void_p(h), ctypes.c_void_p(d_g), ctypes.c_void_p(d_out),
                                     ctypes.c_void_p(stream)), "psflib_apply_adjoint")


def apply_batched(h: int, d_scenes: int, d_images: int, B: int, stream: int):
    _check(_lib.psflib_apply_batched(ctypes.c_void_p(h), ctypes.c_void_p(d_scenes),
                                     ctypes.c_void_p(d_images), ctypes.c_int32(B),
                                     ctypes.c_void_p(stream)), "psflib_apply_batched")


def column_sums(h: int, d_tau: int, stream: int):
    _check(_lib.psflib_column_sums(ctypes.c_void_p(h), ctypes.c_void_p(d_tau), ctypes.c_void_p(stream)),
           "psflib_column_sums")


def get_columns(h: int, d_cols: int, count: int, d_out: int, stream: int):
    _check(_lib.psflib_get_columns(ctypes.c_void_p(h), ctypes.c_void_p(d_cols), ctypes.c_int32(count),
                                   ctypes.c_void_p(d_out), ctypes.c_void_p(stream)),
           "psflib_get_columns")


def get_exponents(h: int, d_exp: int, stream: int):
    _check(_lib.psflib_get_exponents(ctypes.c_void_p(h), ctypes.c_void_p(d_exp), ctypes.c_void_p(stream)),
           "psflib_get_exponents")


def get_geometry(h: int, d_geom: int, d_k: int, stream: int):
    _check(_lib.psflib_get_geometry(ctypes.c_void_p(h), ctypes.c_void_p(d_geom), ctypes.c_void_p(d_k),
                                    ctypes.c_void_p(stream)), "psflib_get_geometry")


def render_disk(N: int, S: float, rmax: float, d_theta: int, d_scene: int, stream: int):
    _check(_lib.psflib_render_disk(ctypes.c_int32(N), ctypes.c_double(S), ctypes.c_double(rmax),
                                   ctypes.c_void_p(d_theta), ctypes.c_void_p(d_scene),
                                   ctypes.c_void_p(stream)), "psflib_render_disk")


def chi2(M: int, K: float, d_image: int, d_data: int, d_var: int, d_loss: int, d_grad: int,
         stream: int):
    _check(_lib.psflib_chi2(ctypes.c_int64(M), ctypes.c_double(K), ctypes.c_void_p(d_image),
                            ctypes.c_void_p(d_data), ctypes.c_void_p(d_var), ctypes.c_void_p(d_loss),
                            ctypes.c_void_p(d_grad), ctypes.c_void_p(stream)), "psflib_chi2")


def render_disk_grad(N: int, S: float, rmax: float, d_theta: int, d_dscene: int, d_dtheta: int,
                     stream: int):
    _check(_lib.psflib_render_disk_grad(ctypes.c_int32(N), ctypes.c_double(S), ctypes.c_double(rmax),
                                        ctypes.c_void_p(d_theta), ctypes.c_void_p(d_dscene),
                                        ctypes.c_void_p(d_dtheta), ctypes.c_void_p(stream)),
           "psflib_render_disk_grad")


def probe_hbm_read(d_buf: int, nbytes: int, workgroups: int, unroll: int, slice: bool,
                   d_sink: int, stream: int):
    _check(_lib.psflib_probe_hbm_read(ctypes.c_void_p(d_buf), ctypes.c_size_t(nbytes),
                                      ctypes.c_int32(workgroups), ctypes.c_int32(unroll),
                                      ctypes.c_int32(1 if slice else 0),
                                      ctypes.c_void_p(d_sink), ctypes.c_void_p(stream)),
           "psflib_probe_hbm_read")


def probe_mfma(kind: int, iters: int, workgroups: int, d_sink: int, stream: int):
    _check(_lib.psflib_probe_mfma(ctypes.c_int32(kind), ctypes.c_int32(iters),
                                  ctypes.c_int32(workgroups), ctypes.c_void_p(d_sink),
                                  ctypes.c_void_p(stream)), "psflib_probe_mfma")


def destroy(h: int):
    _lib.psflib_destroy(ctypes.c_void_p(h))


def grouped_create(handles, lib_of_scene, scene_ptrs, image_ptrs, autotune: bool, stream: int) -> int:
    nl = len(handles)
    B = len(lib_of_scene)
    H = (ctypes.c_void_p * nl)(*handles)
    LS = (ctypes.c_int32 * max(B, 1))(*lib_of_scene)
    SP = (ctypes.c_void_p * max(B, 1))(*scene_ptrs)
    IP = (ctypes.c_void_p * max(B, 1))(*image_ptrs)
    g = ctypes.c_void_p()
    _check(_lib.psflib_grouped_create(H, nl, LS, SP, IP, B, 1 if autotune else 0,
                                      ctypes.c_void_p(stream), ctypes.byref(g)),
           "psflib_grouped_create")
    return int(g.value)


def grouped_run(g: int, stream: int):
    _check(_lib.psflib_grouped_run(ctypes.c_void_p(g), ctypes.c_void_p(stream)), "psflib_grouped_run")


def grouped_chunk(g: int):
    c = ctypes.c_int64(0)
    t = ctypes.c_float(0.0)
    _check(_lib.psflib_grouped_chunk(ctypes.c_void_p(g), ctypes.byref(c), ctypes.byref(t)),
           "psflib_grouped_chunk")
    return int(c.value), float(t.value)


def grouped_shape(g: int):
    """(chunk, rows per item, autotuned ms) of a grouped plan."""
    c = ctypes.c_int64(0)
    r = ctypes.c_int32(0)
    t = ctypes.c_float(0.0)
    _check(_lib.psflib_grouped_shape(ctypes.c_void_p(g), ctypes.byref(c), ctypes.byref(r), ctypes.byref(t)),
           "psflib_grouped_shape")
    return int(c.value), int(r.value), float(t.value)


def grouped_set_shape(g: int, chunk: int, rows: int, stream: int):
    _check(_lib.psflib_grouped_set_shape(ctypes.c_void_p(g), ctypes.c_int64(chunk), ctypes.c_int32(rows),
                                         ctypes.c_void_p(stream)), "psflib_grouped_set_shape")


def grouped_destroy(g: int):
    _lib.psflib_grouped_destroy(ctypes.c_void_p(g))


class Grouped:
    """A grouped simulation plan over several :class:`Library` objects.

    ``scenes[b]`` (float32 CUDA, N_L^2 elements) is simulated with
    ``libs[lib_of_scene[b]]`` into ``images[b]`` (allocated here) by one graph
    launch per :meth:`run`."""

    def __init__(self, libs, lib_of_scene, scenes, autotune=True, stream=None):
        import torch
        self.torch = torch
        self.libs = list(libs)  # keep the libraries alive
        self.scenes = [s.contiguous() for s in scenes]
        self.images = [torch.empty(self.libs[L].M, dtype=torch.float32, device=s.device)
                       for L, s in zip(lib_of_scene, self.scenes)]
        for L, s in zip(lib_of_scene, self.scenes):
            if s.numel() != self.libs[L].ncols or s.dtype != torch.float32:
                raise ValueError("scene size does not match its library")
        st = self._stream(stream)
        self.g = grouped_create([lib.h for lib in self.libs], list(lib_of_scene),
                                [s.data_ptr() for s in self.scenes],
                                [im.data_ptr() for im in self.images], autotune, st)

    def _stream(self, stream):
        if stream is None:
            return self.torch.cuda.current_stream().cuda_stream
        return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)

    def run(self, stream=None):
        grouped_run(self.g, self._stream(stream))
        return self.images

    def chunk(self):
        return grouped_chunk(self.g)

    def shape(self):
        """dict(chunk, rows, tuned_ms): the plan's tile shape (chunk 0 = whole columns)."""
        c, r, t = grouped_shape(self.g)
        return {"chunk": c, "rows": r, "tuned_ms": t}

    def set_shape(self, chunk, rows, stream=None):
        grouped_set_shape(self.g, chunk, rows, self._stream(stream))

    def close(self):
        if getattr(self, "g", None):
            grouped_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------- torch wrapper -----
class Library:
    """A built PSF library on the current GPU.

    ``cube``: float32 CUDA tensor [K][n][n]; ``radii``: K increasing offsets
    (host array); ``N``/``S``: scene side and pixel scale (radii's unit).
    The library buffer is a torch uint8 tensor owned by this object; the build
    is enqueued on the current stream.
    """

    def __init__(self, cube, radii, N: int, S: float, interp="linear", oob="clamp",
                 storage="fp32", stream=None, rotate="bilinear", flux="none"):
        import torch
        if not (isinstance(cube, torch.Tensor) and cube.is_cuda and cube.dtype == torch.float32):
            raise TypeError("cube must be a float32 CUDA tensor [K][n][n]")
        if cube.dim() != 3 or cube.shape[1] != cube.shape[2]:
            raise ValueError("cube must be [K][n][n]")
        self.torch = torch
        self.cube = cube.contiguous()
        self.K, self.n = int(cube.shape[0]), int(cube.shape[1])
        self.N, self.S = int(N), float(S)
        self.storage = storage
        self.radii = np.asarray(radii, dtype=np.float64)
        self.desc = make_desc(self.n, self.K, self.N, self.S, interp, oob, storage, rotate, flux)
        self.nbytes = library_bytes(self.desc)
        self.device = cube.device
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        s = self._stream(stream)
        self.h = build(self.desc, self.cube.data_ptr(), self.radii, self.buf.data_ptr(), self.nbytes, s)
        self.M, self.ncols = self.n * self.n, self.N * self.N

    def _stream(self, stream):
        if stream is None:
            return self.torch.cuda.current_stream(self.device).cuda_stream
        return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)

    def _vec(self, x, size, name):
        t = self.torch
        if not (isinstance(x, t.Tensor) and x.dtype == t.float32 and x.device == self.device
                and x.numel() == size):
            raise ValueError(f"{name} must be a float32 tensor on {self.device} with {size} elements")
        return x.contiguous()

    def _out(self, out, shape, name):
        """A new output tensor, or the caller's `out` after checking that the
        kernels can write all of it and nothing past it."""
        t = self.torch
        if out is None:
            return t.empty(shape, dtype=t.float32, device=self.device)
        numel = 1
        for s in shape:
            numel *= int(s)
        if not (isinstance(out, t.Tensor) and out.dtype == t.float32 and out.device == self.device
                and out.is_contiguous() and out.numel() == numel):
            raise ValueError(f"{name} must be a contiguous float32 tensor on {self.device} with "
                             f"{numel} elements")
        return out

    def apply(self, scene, out=None, stream=None):
        Z = self._vec(scene, self.ncols, "scene")
        out = self._out(out, (self.M,), "out")
        apply(self.h, Z.data_ptr(), out.data_ptr(), self._stream(stream))
        return out

    def apply_adjoint(self, g, out=None, stream=None):
        G = self._vec(g, self.M, "g")
        out = self._out(out, (self.ncols,), "out")
        apply_adjoint(self.h, G.data_ptr(), out.data_ptr(), self._stream(stream))
        return out

    def apply_batched(self, scenes, out=None, stream=None):
        t = self.torch
        if not (isinstance(scenes, t.Tensor) and scenes.dtype == t.float32
                and scenes.device == self.device and scenes.dim() == 2
                and scenes.shape[1] == self.ncols):
            raise ValueError(f"scenes must be a float32 tensor [B][{self.ncols}] on {self.device}")
        Zb = scenes.contiguous()
        B = int(Zb.shape[0])
        out = self._out(out, (B, self.M), "out")
        apply_batched(self.h, Zb.data_ptr(), out.data_ptr(), B, self._stream(stream))
        return out

    def column_sums(self, stream=None):
        out = self.torch.empty(self.ncols, dtype=self.torch.float64, device=self.device)
        column_sums(self.h, out.data_ptr(), self._stream(stream))
        return out

    def get_columns(self, cols, stream=None):
        t = self.torch
        idx = t.as_tensor(np.asarray(cols, dtype=np.int32), device=self.device)
        out = t.empty((idx.numel(), self.M), dtype=t.float32, device=self.device)
        get_columns(self.h, idx.data_ptr(), idx.numel(), out.data_ptr(), self._stream(stream))
        return out

    def exponents(self, stream=None):
        out = self.torch.empty(self.ncols, dtype=self.torch.int32, device=self.device)
        get_exponents(self.h, out.data_ptr(), self._stream(stream))
        return out

    def geometry(self, stream=None):
        t = self.torch
        g = t.empty((self.ncols, 4), dtype=t.float64, device=self.device)
        k = t.empty(self.ncols, dtype=t.int32, device=self.device)
        get_geometry(self.h, g.data_ptr(), k.data_ptr(), self._stream(stream))
        return g, k

    def close(self):
        if getattr(self, "h", None):
            destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
