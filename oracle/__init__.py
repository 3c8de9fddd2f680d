"""ctypes wrapper around the FP64 CPU oracle (oracle/liboracle.so).

TEST INFRASTRUCTURE: imported only by the test suite, the smoke check and the
CPU baseline leg of the benchmark. Fields are numpy complex128 arrays of shape
(nt, nz, ny, nx, 4, 3, 3) in C order (the canonical layout of or.h).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# GF_ORACLE_LIB selects another build of the same source (the sanitizer build
# that a CPU test runs the pins under)
LIB_PATH = os.environ.get("GF_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

LANDAU = 0
COULOMB = 1

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        d = C.POINTER(C.c_double)
        i32p = C.POINTER(C.c_int32)
        u32p = C.POINTER(C.c_uint32)
        i64p = C.POINTER(C.c_int64)
        sig = {
            "or_check_dims": (C.c_int, [i32p]),
            "or_volume": (C.c_int64, [i32p]),
            "or_num_threads": (C.c_int, []),
            "or_set_num_threads": (None, [C.c_int]),
            "or_su2_part": (None, [d, C.c_int, C.c_int, d]),
            "or_overrelax": (C.c_int, [d, C.c_double, d]),
            "or_overrelax_form": (C.c_int, [d, C.c_double, C.c_int, d]),
            "or_mag_matrix": (None, [d, i32p, C.c_int64, C.c_int, d]),
            "or_mag_local_max": (C.c_int, [d, i32p, C.c_int64, C.c_int, d]),
            "or_mag_sweep": (C.c_int, [d, i32p, C.c_int, C.c_double, C.c_int]),
            "or_mag_functional": (C.c_double, [d, i32p]),
            "or_mag_site_gaps": (C.c_int, [d, i32p, C.c_int64, C.c_double, C.c_int, d]),
            "or_mag_theta": (C.c_double, [d, i32p]),
            "or_fix_coulomb_frozen": (C.c_int, [d, i32p, C.c_double, C.c_double, C.c_int32,
                                                C.c_int32, C.c_int32, i32p, d, d, i32p]),
            "or_fix_mag": (C.c_int, [d, i32p, C.c_double, C.c_int, C.c_double, C.c_int32,
                                     C.c_int32, C.c_int32, i32p, d, d]),
            "or_sweep_form": (C.c_int, [d, i32p, C.c_int, C.c_int, C.c_double, C.c_int]),
            "or_local_K": (None, [d, i32p, C.c_int, C.c_int64, d]),
            "or_sweep": (C.c_int, [d, i32p, C.c_int, C.c_int, C.c_double]),
            "or_update_sites": (C.c_int, [d, i32p, C.c_int, C.c_double, i64p, C.c_int64]),
            "or_heatbath_sites": (C.c_int, [d, i32p, C.c_int, C.c_double, C.c_uint64,
                                            C.c_uint64, i64p, C.c_int64]),
            "or_functional": (C.c_double, [d, i32p, C.c_int, d]),
            "or_functional_raw": (C.c_double, [d, i32p, C.c_int]),
            "or_theta_A": (C.c_double, [d, i32p, C.c_int, d]),
            "or_theta_K": (C.c_double, [d, i32p, C.c_int, d]),
            "or_reunitarize": (None, [d, C.c_int64]),
            "or_plaquette": (C.c_double, [d, i32p]),
            "or_unitarity": (C.c_double, [d, i32p]),
            "or_gauge_transform": (C.c_int, [d, i32p, d]),
            "or_fix": (C.c_int, [d, i32p, C.c_int, C.c_double, C.c_int, C.c_double, C.c_int32,
                                 C.c_int32, C.c_int32, i32p, d, d]),
            "or_philox4x32": (None, [u32p, u32p, u32p]),
            "or_kp_draw": (C.c_int, [C.c_double, C.c_uint64, C.c_uint64, C.c_uint64,
                                     C.c_int, d]),
            "or_heatbath_su2": (C.c_int, [C.c_double, C.c_uint64, C.c_uint64, C.c_uint64,
                                          C.c_int, d]),
            "or_heatbath_half": (C.c_int, [d, i32p, C.c_int, C.c_int, C.c_double,
                                           C.c_uint64, C.c_uint64, i64p]),
            "or_micro_half": (C.c_int, [d, i32p, C.c_int, C.c_int]),
            "or_sweep_sr": (C.c_int, [d, i32p, C.c_int, C.c_int, C.c_double, C.c_double,
                                      C.c_uint64, C.c_uint64]),
            "or_anneal_sweep": (C.c_int, [d, i32p, C.c_int, C.c_double, C.c_uint64,
                                          C.c_uint64, C.c_int, i64p]),
            "or_half_sweep_g": (C.c_int, [d, i32p, C.c_int, C.c_int, C.c_int, C.c_double,
                                          C.c_double, C.c_uint64, C.c_uint64, d]),
            "or_heatbath_site_outcomes": (C.c_int, [d, i32p, C.c_int, C.c_double, C.c_uint64,
                                                    C.c_uint64, C.c_int64, C.c_double, C.c_int,
                                                    d, d]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dims(dims):
    a = (C.c_int32 * 4)(*[int(v) for v in dims])
    return a


def _dptr(a):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _field(U):
    assert U.dtype == np.complex128 and U.flags["C_CONTIGUOUS"], "canonical complex128 field"
    return _dptr(U)


def dims_of(U):
    return tuple(int(v) for v in U.shape[:4])


def check_dims(dims):
    return lib().or_check_dims(_dims(dims))


def set_num_threads(n):
    lib().or_set_num_threads(int(n))


def num_threads():
    return lib().or_num_threads()


def su2_part(M, i, j):
    M = np.ascontiguousarray(M, dtype=np.complex128)
    q = np.zeros(4)
    lib().or_su2_part(_dptr(M), int(i), int(j), _dptr(q))
    return q


def overrelax(q, omega):
    q = np.ascontiguousarray(q, dtype=np.float64)
    s = np.zeros(4)
    rc = lib().or_overrelax(_dptr(q), float(omega), _dptr(s))
    return None if rc != 0 else s


def overrelax_form(q, omega, form):
    q = np.ascontiguousarray(q, dtype=np.float64)
    s = np.zeros(4)
    rc = lib().or_overrelax_form(_dptr(q), float(omega), int(form), _dptr(s))
    return None if rc != 0 else s


def sweep_form(U, gauge, parity, omega, form):
    rc = lib().or_sweep_form(_field(U), _dims(dims_of(U)), int(gauge), int(parity), float(omega),
                             int(form))
    if rc != 0:
        raise ValueError("or_sweep_form: bad arguments")


def mag_matrix(U, s, sg):
    M = np.zeros(16)
    lib().or_mag_matrix(_field(U), _dims(dims_of(U)), int(s), int(sg), _dptr(M))
    return M.reshape(4, 4)


def mag_local_max(U, s, sg):
    a = np.zeros(4)
    rc = lib().or_mag_local_max(_field(U), _dims(dims_of(U)), int(s), int(sg), _dptr(a))
    return None if rc != 0 else a


def mag_sweep(U, parity, omega, form=0):
    rc = lib().or_mag_sweep(_field(U), _dims(dims_of(U)), int(parity), float(omega), int(form))
    if rc != 0:
        raise ValueError("or_mag_sweep: bad arguments")


def mag_site_gaps(U, s, omega, form=0):
    gaps = np.zeros(3)
    rc = lib().or_mag_site_gaps(_field(U), _dims(dims_of(U)), int(s), float(omega), int(form),
                                _dptr(gaps))
    if rc != 0:
        raise ValueError("or_mag_site_gaps: bad arguments")
    return gaps


def mag_functional(U):
    return lib().or_mag_functional(_field(U), _dims(dims_of(U)))


def mag_theta(U):
    return lib().or_mag_theta(_field(U), _dims(dims_of(U)))


def fix_coulomb_frozen(U, omega, theta_target, max_sweeps, check_every=100, reunit_at_check=1):
    nt = U.shape[0]
    sw = C.c_int32(0)
    F = np.zeros(nt)
    th = np.zeros(nt)
    fr = np.zeros(nt, dtype=np.int32)
    rc = lib().or_fix_coulomb_frozen(_field(U), _dims(dims_of(U)), float(omega),
                                     float(theta_target), int(max_sweeps), int(check_every),
                                     int(reunit_at_check), C.byref(sw), _dptr(F), _dptr(th),
                                     fr.ctypes.data_as(C.POINTER(C.c_int32)))
    if rc < 0:
        raise ValueError("or_fix_coulomb_frozen: bad arguments")
    return {"converged": rc == 0, "sweeps": sw.value, "F": F, "theta": th, "frozen_at": fr}


def fix_mag(U, omega, theta_target, max_sweeps, check_every=100, reunit_at_check=1, form=0):
    sw = C.c_int32(0)
    F = C.c_double(0.0)
    th = C.c_double(0.0)
    rc = lib().or_fix_mag(_field(U), _dims(dims_of(U)), float(omega), int(form),
                          float(theta_target), int(max_sweeps), int(check_every),
                          int(reunit_at_check), C.byref(sw), C.byref(F), C.byref(th))
    if rc < 0:
        raise ValueError("or_fix_mag: bad arguments")
    return {"converged": rc == 0, "sweeps": sw.value, "F": F.value, "theta": th.value}


def local_K(U, gauge, s):
    K = np.zeros((3, 3), dtype=np.complex128)
    lib().or_local_K(_field(U), _dims(dims_of(U)), int(gauge), int(s), _dptr(K))
    return K


def sweep(U, gauge, parity, omega):
    rc = lib().or_sweep(_field(U), _dims(dims_of(U)), int(gauge), int(parity), float(omega))
    if rc != 0:
        raise ValueError("or_sweep: bad arguments")


def update_sites(U, gauge, omega, sites):
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    rc = lib().or_update_sites(_field(U), _dims(dims_of(U)), int(gauge), float(omega),
                               sites.ctypes.data_as(C.POINTER(C.c_int64)), int(sites.size))
    if rc != 0:
        raise ValueError("or_update_sites: bad arguments")


def heatbath_sites(U, gauge, T, seed, sweep, sites):
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    rc = lib().or_heatbath_sites(_field(U), _dims(dims_of(U)), int(gauge), float(T), int(seed),
                                 int(sweep), sites.ctypes.data_as(C.POINTER(C.c_int64)),
                                 int(sites.size))
    if rc != 0:
        raise ValueError("or_heatbath_sites: bad arguments")


def functional(U, gauge):
    nt = U.shape[0]
    out = np.zeros(nt if gauge == COULOMB else 1)
    v = lib().or_functional(_field(U), _dims(dims_of(U)), int(gauge), _dptr(out))
    return v, out


def functional_raw(U, gauge):
    return lib().or_functional_raw(_field(U), _dims(dims_of(U)), int(gauge))


def theta_A(U, gauge):
    nt = U.shape[0]
    out = np.zeros(nt if gauge == COULOMB else 1)
    v = lib().or_theta_A(_field(U), _dims(dims_of(U)), int(gauge), _dptr(out))
    return v, out


def theta_K(U, gauge):
    nt = U.shape[0]
    out = np.zeros(nt if gauge == COULOMB else 1)
    v = lib().or_theta_K(_field(U), _dims(dims_of(U)), int(gauge), _dptr(out))
    return v, out


def reunitarize(U):
    lib().or_reunitarize(_field(U), int(U.size // 9))


def plaquette(U):
    return lib().or_plaquette(_field(U), _dims(dims_of(U)))


def unitarity(U):
    """max over links and elements of |(U U^dag - 1)_ab| (+inf for NaN)"""
    return lib().or_unitarity(_field(U), _dims(dims_of(U)))


def gauge_transform(U, g):
    g = np.ascontiguousarray(g, dtype=np.complex128)
    assert g.shape == U.shape[:4] + (3, 3)
    rc = lib().or_gauge_transform(_field(U), _dims(dims_of(U)), _dptr(g))
    if rc != 0:
        raise ValueError("or_gauge_transform: bad arguments")


def fix(U, gauge, omega, theta_target, max_sweeps, check_every=100, reunit_at_check=1, form=0):
    sw = C.c_int32(0)
    F = C.c_double(0.0)
    th = C.c_double(0.0)
    rc = lib().or_fix(_field(U), _dims(dims_of(U)), int(gauge), float(omega), int(form),
                      float(theta_target), int(max_sweeps), int(check_every),
                      int(reunit_at_check), C.byref(sw), C.byref(F), C.byref(th))
    if rc < 0:
        raise ValueError("or_fix: bad arguments")
    return {"converged": rc == 0, "sweeps": sw.value, "F": F.value, "theta": th.value}


def philox4x32(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32(c, k, o)
    return [int(v) for v in o]


def kp_draw(alpha, seed, site, sweep, subgroup):
    x = C.c_double(0.0)
    n = lib().or_kp_draw(float(alpha), int(seed), int(site), int(sweep), int(subgroup),
                         C.byref(x))
    return (x.value if n > 0 else None), n


def heatbath_su2(alpha, seed, site, sweep, subgroup):
    X = np.zeros(4)
    n = lib().or_heatbath_su2(float(alpha), int(seed), int(site), int(sweep), int(subgroup),
                              _dptr(X))
    return (X if n > 0 else None), n


def heatbath_half(U, gauge, parity, T, seed, sweep):
    capped = C.c_int64(0)
    rc = lib().or_heatbath_half(_field(U), _dims(dims_of(U)), int(gauge), int(parity),
                                float(T), int(seed), int(sweep), C.byref(capped))
    if rc != 0:
        raise ValueError("or_heatbath_half: bad arguments")
    return capped.value


def sweep_sr(U, gauge, parity, omega, prob, seed, sweep):
    rc = lib().or_sweep_sr(_field(U), _dims(dims_of(U)), int(gauge), int(parity), float(omega),
                           float(prob), int(seed), int(sweep))
    if rc != 0:
        raise ValueError("or_sweep_sr: bad arguments")


def micro_half(U, gauge, parity):
    rc = lib().or_micro_half(_field(U), _dims(dims_of(U)), int(gauge), int(parity))
    if rc != 0:
        raise ValueError("or_micro_half: bad arguments")


def anneal_sweep(U, gauge, T, seed, sweep, n_micro):
    capped = C.c_int64(0)
    rc = lib().or_anneal_sweep(_field(U), _dims(dims_of(U)), int(gauge), float(T), int(seed),
                               int(sweep), int(n_micro), C.byref(capped))
    if rc != 0:
        raise ValueError("or_anneal_sweep: bad arguments")
    return capped.value


# update kinds of half_sweep_g
OR, HEATBATH, MICRO, SR = 0, 1, 2, 3


def half_sweep_g(U, gauge, parity, kind, omega=1.0, param=0.0, seed=0, sweep=0):
    """Half-sweep of the given kind (OR, HEATBATH with param = T, MICRO, SR
    with param = prob) in place; returns g (nt, nz, ny, nx, 3, 3): each updated
    site's total transformation, 1 at the other parity."""
    g = np.zeros(U.shape[:4] + (3, 3), dtype=np.complex128)
    rc = lib().or_half_sweep_g(_field(U), _dims(dims_of(U)), int(gauge), int(parity), int(kind),
                               float(omega), float(param), int(seed), int(sweep), _dptr(g))
    if rc != 0:
        raise ValueError("or_half_sweep_g: bad arguments")
    return g


def heatbath_site_outcomes(U, gauge, T, seed, sweep, s, tau, max_out=64):
    """All results of the heatbath update of site s when the trials whose
    accept margin is below tau may go either way: (outcomes (n, 8, 3, 3)
    complex128 -- U_mu(s) mu = 0..3 then U_mu(s - mu) --, smallest margin on
    the exact path). outcomes[0] is the exact result."""
    out = np.zeros((max_out, 8, 3, 3), dtype=np.complex128)
    mm = C.c_double(0.0)
    n = lib().or_heatbath_site_outcomes(_field(U), _dims(dims_of(U)), int(gauge), float(T),
                                        int(seed), int(sweep), int(s), float(tau), int(max_out),
                                        _dptr(out), C.byref(mm))
    if n < 0:
        raise ValueError("or_heatbath_site_outcomes: bad arguments")
    return out[:n].copy(), mm.value
