"""FP64 CPU oracle for the SU(2) heat-bath path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps the plain C reference in su2_oracle.c with
ctypes and numpy; the arrays it takes and returns use the canonical host
layout U[t][z][y][x][mu][4] (float64), i.e. numpy shape (Nt, Nz, Ny, Nx, 4, 4).

Method and readings: see the header comments of su2_oracle.h / su2_oracle.c.
"""
import ctypes
import os

import numpy as np

from .build import ensure_built

_lib = None

FLAG_CAP = 1
FLAG_NONFINITE = 2
MAX_ATTEMPTS = 4096


def lib():
    global _lib
    if _lib is None:
        path = ensure_built()
        L = ctypes.CDLL(path)
        i4 = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64, u32, i32, i64, dbl = (ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                   ctypes.c_int64, ctypes.c_double)
        sig = {
            "or_philox4x32_10": (None, [u32p, u32p, u32p]),
            "or_u01_f64": (dbl, [u32, u32]),
            "or_u01_f32": (ctypes.c_float, [u32]),
            "or_qmul": (None, [dp, dp, dp]),
            "or_qdag": (None, [dp, dp]),
            "or_volume": (i64, [i4]),
            "or_neighbor": (i64, [i4, i64, i32, i32]),
            "or_parity": (i32, [i4, i64]),
            "or_staple": (None, [i4, dp, i64, i32, dp]),
            "or_init_cold": (None, [i4, dp]),
            "or_init_hot": (None, [i4, dp, u64, u32]),
            "or_heatbath_halfsweep": (u32, [i4, dp, dbl, u64, u32, i32, i32, u32]),
            "or_heatbath_halfsweep_f32": (u32, [i4, dp, dbl, u64, u32, i32, i32, u32]),
            "or_heatbath_sweep": (u32, [i4, dp, dbl, u64, u32, u32]),
            "or_overrelax_halfsweep": (u32, [i4, dp, i32, i32]),
            "or_overrelax_sweep": (u32, [i4, dp]),
            "or_plaquette": (dbl, [i4, dp, dp]),
            "or_polyakov_field": (None, [i4, dp, dp]),
            "or_polyakov": (None, [i4, dp, dp]),
            "or_polyakov_corr": (i32, [i4, dp, dp]),
            "or_gauge_transform": (None, [i4, dp, u64, u32]),
            "or_num_threads": (i32, []),
            "or_bessel_ive": (dbl, [i32, dbl]),
            "or_log_z": (dbl, [dbl]),
            "or_bessel_ratio": (dbl, [dbl]),
            "or_block_colour": (i32, [i32, i32, i32]),
            "or_block_piece": (None, [i4, dp, i64, i32, dp]),
            "or_block_log_marginal": (dbl, [i4, dp, i64, dbl, dp]),
            "or_block_proposal": (None, [i4, dp, i64, dbl, dp, dp]),
            "or_block_move": (u32, [i4, dp, dbl, u64, u32, i32, i32, dp, u32, ctypes.POINTER(ctypes.c_int64)]),
            "or_block_pieces_all": (None, [i4, dp, dp]),
            "or_block_sweep": (u32, [i4, dp, dbl, u64, u32, dp, u32, ctypes.POINTER(ctypes.c_int64)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dims(n):
    n = tuple(int(v) for v in n)
    if len(n) != 4:
        raise ValueError("extents must be (Nx, Ny, Nz, Nt)")
    return (ctypes.c_int * 4)(*n)


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check_links(n, U):
    nx, ny, nz, nt = n
    if U.shape != (nt, nz, ny, nx, 4, 4) or U.dtype != np.float64 or not U.flags.c_contiguous:
        raise ValueError(f"links must be float64 C-contiguous of shape {(nt, nz, ny, nx, 4, 4)}")


def new_links(n):
    nx, ny, nz, nt = n
    return np.zeros((nt, nz, ny, nx, 4, 4), dtype=np.float64)


def num_threads():
    return lib().or_num_threads()


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xffffffff for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def u01_f64(r_even, r_odd):
    return lib().or_u01_f64(r_even & 0xffffffff, r_odd & 0xffffffff)


def u01_f32(r_even):
    return lib().or_u01_f32(r_even & 0xffffffff)


def qmul(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    o = np.empty(4)
    lib().or_qmul(_dp(a), _dp(b), _dp(o))
    return o


def qdag(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    o = np.empty(4)
    lib().or_qdag(_dp(a), _dp(o))
    return o


def neighbor(n, site, direction, step):
    return lib().or_neighbor(_dims(n), site, direction, step)


def parity(n, site):
    return lib().or_parity(_dims(n), site)


def staple(n, U, site, mu):
    _check_links(n, U)
    V = np.empty(4)
    lib().or_staple(_dims(n), _dp(U), site, mu, _dp(V))
    return V


def init_cold(n):
    U = new_links(n)
    lib().or_init_cold(_dims(n), _dp(U))
    return U


def init_hot(n, seed, lattice_id=0):
    U = new_links(n)
    lib().or_init_hot(_dims(n), _dp(U), seed, lattice_id)
    return U


def heatbath_halfsweep(n, U, beta, seed, sweep, mu, parity, lattice_id=0):
    _check_links(n, U)
    return lib().or_heatbath_halfsweep(_dims(n), _dp(U), beta, seed, sweep, mu, parity, lattice_id)


def heatbath_halfsweep_f32(n, U, beta, seed, sweep, mu, parity, lattice_id=0):
    """The half-sweep with single-precision links (U must hold FP32-representable
    values; the updated links are FP32 values): every accept/reject decision
    in the precisions of the single-precision path."""
    _check_links(n, U)
    if not np.array_equal(U.astype(np.float32).astype(np.float64), U):
        raise ValueError("U must hold values representable in single precision")
    return lib().or_heatbath_halfsweep_f32(_dims(n), _dp(U), beta, seed, sweep, mu, parity, lattice_id)


def heatbath_sweep(n, U, beta, seed, sweep, lattice_id=0):
    _check_links(n, U)
    return lib().or_heatbath_sweep(_dims(n), _dp(U), beta, seed, sweep, lattice_id)


def overrelax_halfsweep(n, U, mu, parity):
    _check_links(n, U)
    return lib().or_overrelax_halfsweep(_dims(n), _dp(U), mu, parity)


def overrelax_sweep(n, U):
    _check_links(n, U)
    return lib().or_overrelax_sweep(_dims(n), _dp(U))


def plaquette(n, U):
    """Return (mean plaquette, array of the six plane averages 01,02,03,12,13,23)."""
    _check_links(n, U)
    planes = np.empty(6)
    p = lib().or_plaquette(_dims(n), _dp(U), _dp(planes))
    return p, planes


def polyakov_field(n, U):
    _check_links(n, U)
    nx, ny, nz, nt = n
    L = np.empty((nz, ny, nx))
    lib().or_polyakov_field(_dims(n), _dp(U), _dp(L))
    return L


def polyakov(n, U):
    """Return (spatial mean of L, spatial mean of |L|)."""
    _check_links(n, U)
    out = np.empty(2)
    lib().or_polyakov(_dims(n), _dp(U), _dp(out))
    return float(out[0]), float(out[1])


def polyakov_corr(n, U):
    """Return C(r) for r = 1 .. min(Nx,Ny,Nz)//2."""
    _check_links(n, U)
    C = np.empty(max(1, min(n[:3]) // 2))
    r = lib().or_polyakov_corr(_dims(n), _dp(U), _dp(C))
    return C[:r]


def gauge_transform(n, U, seed, lattice_id=0):
    _check_links(n, U)
    lib().or_gauge_transform(_dims(n), _dp(U), seed, lattice_id)


# ---------------------------------------------------------------------------
# learned block proposal (reference)
# ---------------------------------------------------------------------------
def bessel_ive(order, x):
    return lib().or_bessel_ive(order, x)


def log_z(a):
    """log Z(a) = log(2 I1(a)/a): normalisation of exp(a w0) over Haar measure."""
    return lib().or_log_z(a)


def bessel_ratio(a):
    return lib().or_bessel_ratio(a)


def block_colour(x, y, z):
    return lib().or_block_colour(x, y, z)


def block_piece(n, U, e, direction):
    _check_links(n, U)
    S = np.empty(4)
    lib().or_block_piece(_dims(n), _dp(U), e, direction, _dp(S))
    return S


def block_log_marginal(n, U, e, beta, T):
    _check_links(n, U)
    T = np.ascontiguousarray(T, dtype=np.float64)
    return lib().or_block_log_marginal(_dims(n), _dp(U), e, beta, _dp(T))


def block_proposal(n, U, e, beta, y6):
    _check_links(n, U)
    y6 = np.ascontiguousarray(y6, dtype=np.float64)
    M = np.empty(4)
    lib().or_block_proposal(_dims(n), _dp(U), e, beta, _dp(y6), _dp(M))
    return M


def _y_array(n, y):
    nx, ny, nz, nt = n
    if y is None:
        y = np.zeros((nt, nz, ny, nx, 6))
    y = np.ascontiguousarray(y, dtype=np.float64)
    assert y.shape == (nt, nz, ny, nx, 6)
    return y


def block_move(n, U, beta, seed, step, parity, colour, y=None, lattice_id=0):
    """One class of block moves; y[t, z, y, x, d] network outputs. Returns (flags, accepted)."""
    _check_links(n, U)
    y = _y_array(n, y)
    acc = ctypes.c_int64(0)
    f = lib().or_block_move(_dims(n), _dp(U), beta, seed, step, parity, colour, _dp(y), lattice_id,
                            ctypes.byref(acc))
    return f, acc.value


def block_sweep(n, U, beta, seed, step, y=None, lattice_id=0):
    _check_links(n, U)
    y = _y_array(n, y)
    acc = ctypes.c_int64(0)
    f = lib().or_block_sweep(_dims(n), _dp(U), beta, seed, step, _dp(y), lattice_id, ctypes.byref(acc))
    return f, acc.value


def block_pieces_all(n, U):
    """S[t, z, y, x, d, 4]: the block pieces of every site."""
    _check_links(n, U)
    nx, ny, nz, nt = n
    S = np.empty((nt, nz, ny, nx, 6, 4))
    lib().or_block_pieces_all(_dims(n), _dp(U), _dp(S))
    return S
