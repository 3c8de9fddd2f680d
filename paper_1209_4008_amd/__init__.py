"""Python binding of libgf (MI355X checkerboard overrelaxation gauge fixing).

Argument marshalling only: every step runs in the HIP kernels of libgf.so,
called through its C ABI (include/gf.h). PyTorch is used for device memory and
streams. There is no fallback: if libgf.so is missing or no GPU is present,
the calls raise.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgf.so")

OK, NOT_CONVERGED = 0, 1
ERR_ARG, ERR_UNSUPPORTED, ERR_DEVICE, ERR_HIP, ERR_NONFINITE, ERR_NOMEM = -1, -2, -3, -4, -5, -6
LANDAU, COULOMB, MAG = 0, 1, 2
FP32, FP64 = 4, 8
R12, R18 = 12, 18
FLAG_TIMING, FLAG_GRAPH, FLAG_NO_TRACK, FLAG_FREEZE_TIMESLICES, FLAG_MONITOR = 1, 2, 4, 8, 16


class GFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libgf status {status}: {msg}")
        self.status = status


class Geom(C.Structure):
    _fields_ = [("nt", C.c_int32), ("nz", C.c_int32), ("ny", C.c_int32), ("nx", C.c_int32),
                ("prec", C.c_int32), ("storage", C.c_int32)]

    @classmethod
    def make(cls, dims, prec=FP64, storage=R18):
        nt, nz, ny, nx = (int(v) for v in dims)
        return cls(nt, nz, ny, nx, int(prec), int(storage))

    @property
    def dims(self):
        return (self.nt, self.nz, self.ny, self.nx)

    @property
    def volume(self):
        return self.nt * self.nz * self.ny * self.nx


class CheckRecord(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("prec", C.c_int32), ("F", C.c_double),
                ("theta", C.c_double), ("unitarity", C.c_double), ("elapsed_ms", C.c_double)]

    def as_dict(self):
        return {"sweeps": self.sweeps, "precision": "fp32" if self.prec == FP32 else "fp64",
                "F": self.F, "theta": self.theta, "unitarity": self.unitarity,
                "elapsed_ms": self.elapsed_ms}


class FixParams(C.Structure):
    _fields_ = [("omega", C.c_double), ("theta_target", C.c_double),
                ("theta_switch", C.c_double), ("max_sweeps", C.c_int32),
                ("check_every", C.c_int32), ("reunit_at_check", C.c_int32),
                ("flags", C.c_uint32), ("sa_steps", C.c_int32), ("sa_micro", C.c_int32),
                ("sa_reunit_every", C.c_int32), ("or_form", C.c_int32),
                ("sa_T0", C.c_double), ("sa_T1", C.c_double), ("seed", C.c_uint64),
                ("sr_prob", C.c_double), ("check_log", C.POINTER(CheckRecord)),
                ("check_log_cap", C.c_int32)]


class FixResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("sweeps", C.c_int32), ("sweeps_lo", C.c_int32),
                ("checks", C.c_int32), ("F", C.c_double), ("theta", C.c_double),
                ("theta_at_switch", C.c_double), ("wall_ms", C.c_double),
                ("kernel_ms", C.c_double * 6), ("kernel_launches", C.c_int64 * 6),
                ("sa_steps", C.c_int32), ("frozen_slice_sweeps", C.c_int32),
                ("check_log_n", C.c_int32), ("unitarity_max", C.c_double)]

    def as_dict(self):
        return {"status": self.status, "sweeps": self.sweeps, "sweeps_lo": self.sweeps_lo,
                "checks": self.checks, "F": self.F, "theta": self.theta,
                "theta_at_switch": self.theta_at_switch, "wall_ms": self.wall_ms,
                "kernel_ms": list(self.kernel_ms),
                "kernel_launches": list(self.kernel_launches), "sa_steps": self.sa_steps,
                "frozen_slice_sweeps": self.frozen_slice_sweeps, "check_log_n": self.check_log_n,
                "unitarity_max": self.unitarity_max}


# every symbol of include/gf.h with its ctypes signature
_vp, _gp, _dp = C.c_void_p, C.POINTER(Geom), C.c_void_p
SIGNATURES = {
    "gf_create": (C.c_int32, [C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "gf_destroy": (C.c_int32, [_vp]),
    "gf_last_error": (C.c_char_p, [_vp]),
    "gf_check_geom": (C.c_int32, [_gp]),
    "gf_field_bytes": (C.c_size_t, [_gp]),
    "gf_selftest_host": (C.c_int32, []),
    "gf_version": (C.c_char_p, []),
    "gf_pack": (C.c_int32, [_vp, _gp, _dp, _dp]),
    "gf_unpack": (C.c_int32, [_vp, _gp, _dp, _dp]),
    "gf_convert": (C.c_int32, [_vp, _gp, _dp, _gp, _dp, C.c_int32]),
    "gf_sweep": (C.c_int32, [_vp, _dp, _gp, C.c_int32, C.c_int32, C.c_double]),
    "gf_sweep_form": (C.c_int32, [_vp, _dp, _gp, C.c_int32, C.c_int32, C.c_double, C.c_int32]),
    "gf_sweep_sr": (C.c_int32, [_vp, _dp, _gp, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                C.c_uint64, C.c_uint64]),
    "gf_functional": (C.c_int32, [_vp, _dp, _gp, C.c_int32, _dp]),
    "gf_theta": (C.c_int32, [_vp, _dp, _gp, C.c_int32, _dp]),
    "gf_measure": (C.c_int32, [_vp, _dp, _gp, C.c_int32, _dp, _dp]),
    "gf_measure_static": (C.c_int32, [_vp, _dp, _gp, C.c_int32, _dp, _dp]),
    "gf_unitarity": (C.c_int32, [_vp, _dp, _gp, _dp]),
    "gf_reunitarize": (C.c_int32, [_vp, _dp, _gp]),
    "gf_plaquette": (C.c_int32, [_vp, _dp, _gp, _dp]),
    "gf_heatbath_half": (C.c_int32, [_vp, _dp, _gp, C.c_int32, C.c_int32, C.c_double,
                                     C.c_uint64, C.c_uint64]),
    "gf_micro_half": (C.c_int32, [_vp, _dp, _gp, C.c_int32, C.c_int32]),
    "gf_anneal_sweep": (C.c_int32, [_vp, _dp, _gp, C.c_int32, C.c_double, C.c_uint64,
                                    C.c_uint64, C.c_int32]),
    "gf_philox": (C.c_int32, [_vp, _dp, C.c_uint64, _dp, C.c_int64]),
    "gf_gauge_bytes": (C.c_size_t, [_gp]),
    "gf_gauge_unit": (C.c_int32, [_vp, _gp, _dp]),
    "gf_gauge_pack": (C.c_int32, [_vp, _gp, _dp, _dp]),
    "gf_gauge_unpack": (C.c_int32, [_vp, _gp, _dp, _dp]),
    "gf_sweep_tracked": (C.c_int32, [_vp, _dp, _dp, _gp, C.c_int32, C.c_int32, C.c_double]),
    "gf_heatbath_half_tracked": (C.c_int32, [_vp, _dp, _dp, _gp, C.c_int32, C.c_int32,
                                             C.c_double, C.c_uint64, C.c_uint64]),
    "gf_micro_half_tracked": (C.c_int32, [_vp, _dp, _dp, _gp, C.c_int32, C.c_int32]),
    "gf_set_sweep_variant": (C.c_int32, [_vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "gf_get_sweep_variant": (C.c_int32, [_vp, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int32)]),
    "gf_sweep_variant_for": (C.c_int32, [_vp, _gp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "gf_set_anneal_variant": (C.c_int32, [_vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "gf_anneal_variant_for": (C.c_int32, [_vp, _gp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "gf_autotune": (C.c_int32, [_vp, _gp, C.c_int32, _dp, C.POINTER(C.c_int32),
                                C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
    "gf_autotune_anneal": (C.c_int32, [_vp, _gp, C.c_int32, _dp, C.c_double, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
    "gf_autotune_storage": (C.c_int32, [_vp, _gp, C.c_int32, _dp, C.POINTER(C.c_int32),
                                        C.POINTER(C.c_float)]),
    "gf_stream_probe": (C.c_int32, [_vp, _dp, _dp, C.c_size_t, C.c_int32]),
    "gf_fix": (C.c_int32, [_vp, _dp, _gp, C.c_int32, C.POINTER(FixParams),
                           C.POINTER(FixResult)]),
    "gf_fix_mixed": (C.c_int32, [_vp, _dp, _gp, _dp, _gp, C.c_int32, C.POINTER(FixParams),
                                 C.POINTER(FixResult)]),
    "gf_batch_create": (C.c_int32, [_vp, C.c_int32, C.POINTER(Geom), C.POINTER(C.c_void_p),
                                    C.c_int32, C.POINTER(C.c_void_p)]),
    "gf_batch_run": (C.c_int32, [_vp, C.POINTER(FixParams), C.POINTER(FixResult)]),
    "gf_batch_autotune": (C.c_int32, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_float)]),
    "gf_batch_destroy": (C.c_int32, [_vp]),
}

_lib = None


def lib():
    """Load libgf.so (built by paper_1209_4008_amd/build.py). PyTorch's own HIP
    runtime is started first: with a library built against the system ROCm
    loaded into the process before it, gf_create finds no GPU."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_1209_4008_amd/build.py")
        import torch
        torch.cuda.is_available()
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def field_bytes(geom):
    return int(lib().gf_field_bytes(C.byref(geom)))


def gauge_bytes(geom):
    return int(lib().gf_gauge_bytes(C.byref(geom)))


def check_geom(geom):
    return int(lib().gf_check_geom(C.byref(geom)))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """A libgf context on the current CUDA(HIP) device and torch stream."""

    def __init__(self, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise GFError(ERR_DEVICE, "no GPU available (libgf has no CPU path)")
        self.torch = torch
        if device is None:
            device = torch.cuda.current_device()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        st = lib().gf_create(int(device), C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != OK:
            raise GFError(st, lib().gf_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().gf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow=(OK,)):
        if st not in allow:
            raise GFError(st, lib().gf_last_error(self.h).decode())
        return st

    # ---- memory helpers (torch as allocator) -------------------------------
    def empty_field(self, geom):
        n = field_bytes(geom)
        if n == 0:
            raise GFError(ERR_ARG, "invalid geometry")
        return self.torch.empty(n, dtype=self.torch.uint8, device="cuda")

    def empty_gauge(self, geom):
        n = gauge_bytes(geom)
        if n == 0:
            raise GFError(ERR_ARG, "invalid geometry")
        return self.torch.empty(n, dtype=self.torch.uint8, device="cuda")

    def empty_out(self, n):
        return self.torch.zeros(n, dtype=self.torch.float64, device="cuda")

    # ---- C ABI calls --------------------------------------------------------
    def pack(self, geom, U_canon, U):
        return self._check(lib().gf_pack(self.h, C.byref(geom), _ptr(U_canon), _ptr(U)))

    def unpack(self, geom, U, U_canon):
        return self._check(lib().gf_unpack(self.h, C.byref(geom), _ptr(U), _ptr(U_canon)))

    def convert(self, gsrc, Usrc, gdst, Udst, reunitarize=True):
        return self._check(lib().gf_convert(self.h, C.byref(gsrc), _ptr(Usrc), C.byref(gdst),
                                            _ptr(Udst), int(bool(reunitarize))))

    def sweep(self, U, geom, gauge, parity, omega):
        return self._check(lib().gf_sweep(self.h, _ptr(U), C.byref(geom), int(gauge),
                                          int(parity), float(omega)))

    def sweep_form(self, U, geom, gauge, parity, omega, form):
        return self._check(lib().gf_sweep_form(self.h, _ptr(U), C.byref(geom), int(gauge),
                                               int(parity), float(omega), int(form)))

    def sweep_sr(self, U, geom, gauge, parity, omega, prob, seed, sweep):
        return self._check(lib().gf_sweep_sr(self.h, _ptr(U), C.byref(geom), int(gauge),
                                             int(parity), float(omega), float(prob), int(seed),
                                             int(sweep)))

    def measure(self, U, geom, gauge, F=None, theta=None):
        return self._check(lib().gf_measure(self.h, _ptr(U), C.byref(geom), int(gauge),
                                            _ptr(F), _ptr(theta)))

    def measure_static(self, U, geom, gauge, F=None, theta=None):
        return self._check(lib().gf_measure_static(self.h, _ptr(U), C.byref(geom), int(gauge),
                                                   _ptr(F), _ptr(theta)))

    def unitarity(self, U, geom, out):
        """largest |U U^dag - 1| element over all links into out (1 device double)"""
        return self._check(lib().gf_unitarity(self.h, _ptr(U), C.byref(geom), _ptr(out)))

    def functional(self, U, geom, gauge, F):
        return self._check(lib().gf_functional(self.h, _ptr(U), C.byref(geom), int(gauge),
                                               _ptr(F)))

    def theta(self, U, geom, gauge, th):
        return self._check(lib().gf_theta(self.h, _ptr(U), C.byref(geom), int(gauge), _ptr(th)))

    def reunitarize(self, U, geom):
        return self._check(lib().gf_reunitarize(self.h, _ptr(U), C.byref(geom)))

    def plaquette(self, U, geom, P):
        return self._check(lib().gf_plaquette(self.h, _ptr(U), C.byref(geom), _ptr(P)))

    def heatbath_half(self, U, geom, gauge, parity, T, seed, sweep):
        return self._check(lib().gf_heatbath_half(self.h, _ptr(U), C.byref(geom), int(gauge),
                                                  int(parity), float(T), int(seed), int(sweep)))

    def micro_half(self, U, geom, gauge, parity):
        return self._check(lib().gf_micro_half(self.h, _ptr(U), C.byref(geom), int(gauge),
                                               int(parity)))

    def anneal_sweep(self, U, geom, gauge, T, seed, sweep, n_micro):
        return self._check(lib().gf_anneal_sweep(self.h, _ptr(U), C.byref(geom), int(gauge),
                                                 float(T), int(seed), int(sweep), int(n_micro)))

    def gauge_unit(self, geom, G):
        return self._check(lib().gf_gauge_unit(self.h, C.byref(geom), _ptr(G)))

    def gauge_pack(self, geom, g_canon, G):
        return self._check(lib().gf_gauge_pack(self.h, C.byref(geom), _ptr(g_canon), _ptr(G)))

    def gauge_unpack(self, geom, G, g_canon):
        return self._check(lib().gf_gauge_unpack(self.h, C.byref(geom), _ptr(G), _ptr(g_canon)))

    def sweep_tracked(self, U, G, geom, gauge, parity, omega):
        return self._check(lib().gf_sweep_tracked(self.h, _ptr(U), _ptr(G), C.byref(geom),
                                                  int(gauge), int(parity), float(omega)))

    def heatbath_half_tracked(self, U, G, geom, gauge, parity, T, seed, sweep):
        return self._check(lib().gf_heatbath_half_tracked(self.h, _ptr(U), _ptr(G), C.byref(geom),
                                                          int(gauge), int(parity), float(T),
                                                          int(seed), int(sweep)))

    def micro_half_tracked(self, U, G, geom, gauge, parity):
        return self._check(lib().gf_micro_half_tracked(self.h, _ptr(U), _ptr(G), C.byref(geom),
                                                       int(gauge), int(parity)))

    def philox(self, ctr, seed, out, n):
        return self._check(lib().gf_philox(self.h, _ptr(ctr), int(seed), _ptr(out), int(n)))

    def set_sweep_variant(self, prec, storage, tps=0, nontemporal=-1):
        return self._check(lib().gf_set_sweep_variant(self.h, int(prec), int(storage), int(tps),
                                                      int(nontemporal)))

    def get_sweep_variant(self, prec, storage):
        t, n = C.c_int32(0), C.c_int32(0)
        self._check(lib().gf_get_sweep_variant(self.h, int(prec), int(storage), C.byref(t),
                                               C.byref(n)))
        return t.value, n.value

    def sweep_variant_for(self, geom):
        t, n = C.c_int32(0), C.c_int32(0)
        self._check(lib().gf_sweep_variant_for(self.h, C.byref(geom), C.byref(t), C.byref(n)))
        return t.value, n.value

    def autotune(self, geom, gauge=LANDAU, U_like=None):
        """Time the nine sweep variants (lanes per site 1, 2, 4 x nontemporal
        mode 0 none, 1 loads and stores, 2 stores only) for geom on a copy of
        U_like (None: the unit field); keep the fastest on this context.
        Returns ((tps, nontemporal), {(tps, nontemporal): ms per half-sweep})."""
        t, n = C.c_int32(0), C.c_int32(0)
        ms = (C.c_float * 9)()
        self._check(lib().gf_autotune(self.h, C.byref(geom), int(gauge), _ptr(U_like),
                                      C.byref(t), C.byref(n), ms))
        table = {(1 << (k % 3), k // 3): ms[k] for k in range(9)}
        return (t.value, n.value), table

    def autotune_anneal(self, geom, gauge, U_like=None, T=1.0):
        """The same for the annealing updates at temperature T."""
        t, n = C.c_int32(0), C.c_int32(0)
        ms = (C.c_float * 9)()
        self._check(lib().gf_autotune_anneal(self.h, C.byref(geom), int(gauge), _ptr(U_like),
                                             float(T), C.byref(t), C.byref(n), ms))
        table = {(1 << (k % 3), k // 3): ms[k] for k in range(9)}
        return (t.value, n.value), table

    def autotune_storage(self, geom, gauge, U_canon):
        """Storage axis: (GF_R12 or GF_R18, {R12: ms, R18: ms}) per half-sweep of
        each storage's best variant for geom's extents and precision."""
        st = C.c_int32(0)
        ms = (C.c_float * 2)()
        self._check(lib().gf_autotune_storage(self.h, C.byref(geom), int(gauge), _ptr(U_canon),
                                              C.byref(st), ms))
        return st.value, {R12: ms[0], R18: ms[1]}

    def set_anneal_variant(self, prec, storage, tps=0, nontemporal=-1):
        return self._check(lib().gf_set_anneal_variant(self.h, int(prec), int(storage), int(tps),
                                                       int(nontemporal)))

    def anneal_variant_for(self, geom):
        t, n = C.c_int32(0), C.c_int32(0)
        self._check(lib().gf_anneal_variant_for(self.h, C.byref(geom), C.byref(t), C.byref(n)))
        return t.value, n.value

    def stream_probe(self, src, dst, nbytes, kind):
        return self._check(lib().gf_stream_probe(self.h, _ptr(src), _ptr(dst), int(nbytes),
                                                 int(kind)))

    def fix(self, U, geom, gauge, params):
        r = FixResult()
        self._check(lib().gf_fix(self.h, _ptr(U), C.byref(geom), int(gauge), C.byref(params),
                                 C.byref(r)), allow=(OK, NOT_CONVERGED))
        return r

    def fix_mixed(self, U_lo, geom_lo, U_hi, geom_hi, gauge, params):
        r = FixResult()
        self._check(lib().gf_fix_mixed(self.h, _ptr(U_lo), C.byref(geom_lo), _ptr(U_hi),
                                       C.byref(geom_hi), int(gauge), C.byref(params),
                                       C.byref(r)), allow=(OK, NOT_CONVERGED))
        return r


class Batch:
    """n independent Landau problems (FP64 fields, uneven extents allowed) fixed
    together by gf_batch_run; the fields are borrowed until close()."""

    def __init__(self, ctx, geoms, fields, gauge=LANDAU):
        self.ctx = ctx
        self.n = len(geoms)
        self.fields = list(fields)  # keep the tensors alive
        ga = (Geom * self.n)(*geoms)
        ua = (C.c_void_p * self.n)(*[f.data_ptr() for f in fields])
        h = C.c_void_p()
        ctx._check(lib().gf_batch_create(ctx.h, self.n, ga, ua, int(gauge), C.byref(h)))
        self.h = h

    def autotune(self):
        """gf_batch_autotune: ((tps, nt) of the FP32 phase, (tps, nt) of the FP64
        phase, {(phase, tps, nt): ms per half-sweep})"""
        tps = (C.c_int32 * 2)()
        nt = (C.c_int32 * 2)()
        ms = (C.c_float * 18)()
        self.ctx._check(lib().gf_batch_autotune(self.h, tps, nt, ms))
        times = {(ph, 1 << (k % 3), k // 3): ms[9 * ph + k] for ph in range(2) for k in range(9)}
        return (tps[0], nt[0]), (tps[1], nt[1]), times

    def run(self, params):
        res = (FixResult * self.n)()
        self.ctx._check(lib().gf_batch_run(self.h, C.byref(params), res),
                        allow=(OK, NOT_CONVERGED))
        return list(res)

    def close(self):
        if getattr(self, "h", None):
            lib().gf_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fix_params(omega=1.7, theta_target=1e-14, theta_switch=1e-6, max_sweeps=20000,
               check_every=100, reunit_at_check=1, flags=0, sa_steps=0, sa_micro=3,
               sa_reunit_every=10, sa_T0=1.45, sa_T1=0.01, seed=0, sr_prob=0.0, or_form=0,
               check_log=None):
    """check_log: None or a (CheckRecord * n)() array the drivers fill, one
    record per check (kept alive by the returned params)"""
    p = FixParams(float(omega), float(theta_target), float(theta_switch), int(max_sweeps),
                  int(check_every), int(reunit_at_check), int(flags), int(sa_steps),
                  int(sa_micro), int(sa_reunit_every), int(or_form), float(sa_T0),
                  float(sa_T1), int(seed), float(sr_prob))
    if check_log is not None:
        p.check_log = C.cast(check_log, C.POINTER(CheckRecord))
        p.check_log_cap = len(check_log)
        p._check_log = check_log
    return p


def check_log(n):
    """an empty log of n check records for fix_params(check_log=...)"""
    return (CheckRecord * int(n))()
