"""Seeded synthetic SU(3) gauge fields (inputs for tests and benchmarks).

This module makes inputs only and holds none of the gauge-fixing arithmetic.
Host generators fill numpy complex128 arrays of shape (nt, nz, ny, nx, 4, 3, 3)
(canonical layout); device generators fill torch float64 CUDA tensors of the
same number of reals in the same layout. Host and device entry points draw the
same Philox4x32-10 numbers, so they produce the same field from the same seed.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgfinputs.so")

_lib = None


def _torch_hip_first():
    """PyTorch carries its own HIP runtime. If this library, built against the
    system ROCm, is loaded into a process first, libgf later finds no GPU
    (gf_create: no GPU device available), so torch's runtime is started
    before the library is loaded (on a machine without a GPU this only asks
    torch, which answers no)."""
    import torch
    torch.cuda.is_available()


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _torch_hip_first()
        L = C.CDLL(LIB_PATH)
        d = C.POINTER(C.c_double)
        i32p = C.POINTER(C.c_int32)
        u32p = C.POINTER(C.c_uint32)
        sig = {
            "gen_unit_field": (C.c_int, [d, i32p]),
            "gen_haar_sites": (C.c_int, [d, i32p, C.c_uint64, C.c_uint32]),
            "gen_smooth_links": (C.c_int, [d, i32p, C.c_double, C.c_uint64]),
            "gen_config0": (C.c_int, [d, i32p, C.c_double, C.c_uint64]),
            "gen_pure_gauge": (C.c_int, [d, i32p, C.c_uint64]),
            "gen_haar_copy": (C.c_int, [d, i32p, C.c_uint64, C.c_uint32]),
            "gen_heatbath_sweep": (C.c_int, [d, i32p, C.c_double, C.c_uint64, C.c_uint32]),
            "gen_philox4x32": (None, [u32p, u32p, u32p]),
            "gen_gpu_unit_field": (C.c_int, [C.c_void_p, i32p, C.c_void_p]),
            "gen_gpu_config0": (C.c_int, [C.c_void_p, i32p, C.c_double, C.c_uint64,
                                          C.c_void_p]),
            "gen_gpu_haar_copy": (C.c_int, [C.c_void_p, i32p, C.c_uint64, C.c_uint32,
                                            C.c_void_p]),
            "gen_gpu_config0_packed": (C.c_int, [C.c_void_p, i32p, C.c_int32, C.c_int32,
                                                 C.c_double, C.c_uint64, C.c_void_p]),
            "gen_gpu_heatbath_sweep": (C.c_int, [C.c_void_p, i32p, C.c_double, C.c_uint64,
                                                 C.c_uint32, C.c_void_p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dims(dims):
    return (C.c_int32 * 4)(*[int(v) for v in dims])


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed with status {rc}")


def empty_field(dims):
    return np.zeros(tuple(dims) + (4, 3, 3), dtype=np.complex128)


def unit_field(dims):
    U = empty_field(dims)
    _check(lib().gen_unit_field(_dp(U), _dims(dims)), "gen_unit_field")
    return U


def haar_sites(dims, seed, copy=0):
    g = np.zeros(tuple(dims) + (3, 3), dtype=np.complex128)
    _check(lib().gen_haar_sites(_dp(g), _dims(dims), int(seed), int(copy)), "gen_haar_sites")
    return g


def smooth_links(dims, eps, seed):
    U = empty_field(dims)
    _check(lib().gen_smooth_links(_dp(U), _dims(dims), float(eps), int(seed)), "gen_smooth_links")
    return U


def config0(dims=(8, 8, 8, 8), eps=0.3, seed=1):
    """exp(i eps H) links hit by a Haar gauge transformation (all from `seed`)."""
    U = empty_field(dims)
    _check(lib().gen_config0(_dp(U), _dims(dims), float(eps), int(seed)), "gen_config0")
    return U


def pure_gauge(dims, seed):
    U = empty_field(dims)
    _check(lib().gen_pure_gauge(_dp(U), _dims(dims), int(seed)), "gen_pure_gauge")
    return U


def abelian_gauge(dims, seed, eps=0.5):
    """Diagonal SU(3) links diag(e^{i t1}, e^{i t2}, e^{-i(t1+t2)}), t uniform in
    [-eps pi, eps pi] (numpy Philox stream `seed`), hit by a Haar gauge
    transformation (gen_haar_copy with `seed`, copy 0): a gauge copy of an
    Abelian field."""
    rng = np.random.Generator(np.random.Philox(int(seed)))
    t = rng.uniform(-eps * np.pi, eps * np.pi, size=tuple(dims) + (4, 2))
    U = np.zeros(tuple(dims) + (4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = np.exp(1j * t[..., 0])
    U[..., 1, 1] = np.exp(1j * t[..., 1])
    U[..., 2, 2] = np.exp(-1j * (t[..., 0] + t[..., 1]))
    return haar_copy(U, seed, 0)


def abelian_noise(dims, seed, eps):
    """diag(e^{i t1}, e^{i t2}, e^{-i(t1+t2)}) exp(i eps H) per link: random
    diagonal phases (t uniform in [-pi, pi], numpy Philox stream `seed`) times
    the links of smooth_links(dims, eps, seed); close to the maximally Abelian
    gauge without being in it."""
    rng = np.random.Generator(np.random.Philox(int(seed)))
    t = rng.uniform(-np.pi, np.pi, size=tuple(dims) + (4, 2))
    V = smooth_links(dims, eps, seed)
    d = np.stack([np.exp(1j * t[..., 0]), np.exp(1j * t[..., 1]),
                  np.exp(-1j * (t[..., 0] + t[..., 1]))], axis=-1)
    return np.ascontiguousarray(d[..., :, None] * V)


def haar_copy(U, seed, copy):
    """In place: U_mu(x) <- h(x) U_mu(x) h(x+mu)^dag with Haar h from (seed, copy)."""
    assert U.dtype == np.complex128 and U.flags["C_CONTIGUOUS"]
    _check(lib().gen_haar_copy(_dp(U), _dims(U.shape[:4]), int(seed), int(copy)),
           "gen_haar_copy")
    return U


def heatbath(dims, beta, sweeps, seed, U=None, first_sweep=0):
    """Quenched Wilson-action heatbath on the host (small lattices), cold start."""
    if U is None:
        U = unit_field(dims)
    for k in range(sweeps):
        _check(lib().gen_heatbath_sweep(_dp(U), _dims(dims), float(beta), int(seed),
                                        int(first_sweep + k)), "gen_heatbath_sweep")
    return U


def philox4x32(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().gen_philox4x32(c, k, o)
    return [int(v) for v in o]


# ---- device generators (torch CUDA tensors; torch is only the allocator) ------------

def _stream_ptr(torch):
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def device_field(dims, torch):
    V = int(np.prod(dims))
    return torch.empty(V * 4 * 18, dtype=torch.float64, device="cuda")


def gpu_unit_field(dims):
    import torch
    U = device_field(dims, torch)
    _check(lib().gen_gpu_unit_field(C.c_void_p(U.data_ptr()), _dims(dims), _stream_ptr(torch)),
           "gen_gpu_unit_field")
    return U


def gpu_config0(dims, eps=0.3, seed=1):
    import torch
    U = device_field(dims, torch)
    _check(lib().gen_gpu_config0(C.c_void_p(U.data_ptr()), _dims(dims), float(eps), int(seed),
                                 _stream_ptr(torch)), "gen_gpu_config0")
    return U


def gpu_config0_packed(F, dims, prec_bytes, nc, eps=0.3, seed=1):
    """gpu_config0's links, rounded to float (prec_bytes 4) or double (8), written
    into the gauge-fixing library's tiled device layout with nc = 6 (rows 0 and
    1) or 9 complex per link; F is a CUDA tensor of the field's size in bytes."""
    import torch
    _check(lib().gen_gpu_config0_packed(C.c_void_p(F.data_ptr()), _dims(dims), int(prec_bytes),
                                        int(nc), float(eps), int(seed), _stream_ptr(torch)),
           "gen_gpu_config0_packed")
    return F


def gpu_haar_copy(U, dims, seed, copy):
    import torch
    _check(lib().gen_gpu_haar_copy(C.c_void_p(U.data_ptr()), _dims(dims), int(seed), int(copy),
                                   _stream_ptr(torch)), "gen_gpu_haar_copy")
    return U


def gpu_heatbath(dims, beta, sweeps, seed, U=None, first_sweep=0, progress=None):
    """Quenched Wilson-action heatbath on the device, cold start unless U is given."""
    import torch
    if U is None:
        U = gpu_unit_field(dims)
    for k in range(sweeps):
        _check(lib().gen_gpu_heatbath_sweep(C.c_void_p(U.data_ptr()), _dims(dims), float(beta),
                                            int(seed), int(first_sweep + k), _stream_ptr(torch)),
               "gen_gpu_heatbath_sweep")
        if progress is not None and (k + 1) % progress == 0:
            torch.cuda.synchronize()
            print(f"[inputs] heatbath {dims} beta={beta}: sweep {k + 1}/{sweeps}", flush=True)
    return U
