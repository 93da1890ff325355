"""SU(2) lattice gauge configurations on an MI355X: Python binding of libsu2.so.

The functions below carry the names of the C ABI in include/su2.h and only
marshal arguments: every step of the heat bath, overrelaxation and the
observables runs in the library's HIP kernels.  PyTorch provides device
memory (uint8 tensors) and the current HIP stream.  Importing this package
raises ImportError when libsu2.so has not been built; there is no fallback.

Method: Cardoso, Cardoso & Bicudo, "Finite temperature lattice QCD with
GPUs" (Excited QCD 2011), Sec. 2.1 (random start, heat-bath sweeps, mean
plaquette per sweep) and Sec. 2.2, eqs. (1) and (3) (Polyakov loop and its
correlator).
"""
import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsu2.so")

SU2_F64, SU2_F32 = 0, 1
SU2_OK, SU2_EINVAL, SU2_EDIMS, SU2_EALIGN, SU2_EWORK, SU2_EHIP = 0, -1, -2, -3, -4, -5
SU2_FLAG_CAP, SU2_FLAG_NONFINITE = 1, 2
SU2_MAX_ATTEMPTS = 4096

_PRECS = {"f64": SU2_F64, "f32": SU2_F32, SU2_F64: SU2_F64, SU2_F32: SU2_F32}


class su2_lattice_t(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 4),
        ("prec", ctypes.c_int32),
        ("lattice_id", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("tile_y", ctypes.c_int32),
        ("links", ctypes.c_void_p),
        ("work", ctypes.c_void_p),
        ("work_bytes", ctypes.c_uint64),
    ]


class Su2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_LP = ctypes.POINTER(su2_lattice_t)
_I4 = ctypes.POINTER(ctypes.c_int32)
_VP = ctypes.c_void_p
_SIGNATURES = {
    "su2_links_bytes": (ctypes.c_uint64, [_I4, ctypes.c_int32]),
    "su2_plane_stride": (ctypes.c_uint64, [_I4, ctypes.c_int32]),
    "su2_workspace_bytes": (ctypes.c_uint64, [_I4, ctypes.c_int32]),
    "su2_init_cold": (ctypes.c_int, [_LP, _VP]),
    "su2_init_hot": (ctypes.c_int, [_LP, ctypes.c_uint64, _VP]),
    "su2_heatbath_sweep": (ctypes.c_int, [_LP, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32, _VP]),
    "su2_heatbath_halfsweep": (ctypes.c_int, [_LP, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                              ctypes.c_int32, ctypes.c_int32, _VP]),
    "su2_overrelax": (ctypes.c_int, [_LP, ctypes.c_int32, _VP]),
    "su2_overrelax_halfsweep": (ctypes.c_int, [_LP, ctypes.c_int32, ctypes.c_int32, _VP]),
    "su2_plaquette": (ctypes.c_int, [_LP, _VP, _VP]),
    "su2_plaquette_noalloc": (ctypes.c_int, [_LP, _VP, _VP]),
    "su2_polyakov": (ctypes.c_int, [_LP, _VP, _VP, _VP]),
    "su2_measure": (ctypes.c_int, [_LP, _VP, _VP, _VP, _VP]),
    "su2_heatbath_sweep_measured": (ctypes.c_int, [_LP, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32, _VP,
                                                   _VP]),
    "su2_overrelax_measured": (ctypes.c_int, [_LP, ctypes.c_int32, _VP, _VP]),
    "su2_get_flags": (ctypes.c_int, [_LP, _VP, _VP]),
    "su2_batch_table_bytes": (ctypes.c_uint64, [ctypes.c_int32]),
    "su2_batch_fill": (ctypes.c_int, [_LP, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, _VP, ctypes.c_uint64]),
    "su2_batch_heatbath_sweep": (ctypes.c_int, [_LP, ctypes.c_int32, _VP, ctypes.c_uint64, ctypes.c_uint32, _VP,
                                                _VP]),
    "su2_batch_overrelax": (ctypes.c_int, [_LP, ctypes.c_int32, _VP, ctypes.c_int32, _VP]),
    "su2_batch_polyakov": (ctypes.c_int, [_LP, ctypes.c_int32, _VP, _VP, _VP, ctypes.c_int32, _VP]),
    "su2_batch_sweep": (ctypes.c_int, [_LP, ctypes.c_int32, _VP, ctypes.c_uint64, ctypes.c_uint32, _VP,
                                       ctypes.c_int32, _VP, ctypes.c_uint32, _VP]),
    "su2_sweep_advance": (ctypes.c_int, [_VP, _VP]),
    "su2_lp_param_count": (ctypes.c_int32, []),
    "su2_lp_workspace_bytes": (ctypes.c_uint64, [_I4]),
    "su2_lp_forward": (ctypes.c_int, [_LP, _VP, _VP, ctypes.c_uint64, _VP, _VP]),
    "su2_lp_loss_grad": (ctypes.c_int, [_LP, ctypes.c_double, _VP, _VP, ctypes.c_uint64, _VP, _VP, _VP]),
    "su2_lp_adam": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_float, ctypes.c_float, _VP]),
    "su2_lp_move": (ctypes.c_int, [_LP, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32,
                                   ctypes.c_int32, _VP, _VP, _VP]),
    "su2_lp_sweep": (ctypes.c_int, [_LP, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32, _VP, _VP, _VP]),
    "su2_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "su2_last_error": (ctypes.c_char_p, []),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run `python paper_1104_5432_amd/build.py` "
            "(hipcc for gfx950). There is no CPU fallback.")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(rc):
    if rc != SU2_OK:
        raise Su2Error(rc, f"{lib.su2_strerror(rc).decode()}: {lib.su2_last_error().decode()}")


def _dims(n):
    n = tuple(int(v) for v in n)
    if len(n) != 4:
        raise ValueError("extents must be (Nx, Ny, Nz, Nt)")
    return n, (ctypes.c_int32 * 4)(*n)


def su2_links_bytes(n, prec):
    return int(lib.su2_links_bytes(_dims(n)[1], _PRECS[prec]))


def su2_plane_stride(n, prec):
    return int(lib.su2_plane_stride(_dims(n)[1], _PRECS[prec]))


def su2_workspace_bytes(n, prec):
    return int(lib.su2_workspace_bytes(_dims(n)[1], _PRECS[prec]))


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


class Lattice:
    """Device storage for one lattice: links and workspace as uint8 tensors,
    plus the su2_lattice_t descriptor that points at them."""

    def __init__(self, n, prec="f64", device="cuda", lattice_id=0, tile=0, tile_y=0):
        self.n, cn = _dims(n)
        self.prec = _PRECS[prec]
        nb = su2_links_bytes(self.n, self.prec)
        wb = su2_workspace_bytes(self.n, self.prec)
        if nb == 0 or wb == 0:
            raise Su2Error(SU2_EDIMS, "extents must be even, >= 2, with volume < 2^32")
        self.device = torch.device(device)
        self.links = torch.empty(nb, dtype=torch.uint8, device=self.device)
        self.work = torch.zeros(wb, dtype=torch.uint8, device=self.device)
        self.desc = su2_lattice_t(cn, self.prec, int(lattice_id), int(tile), int(tile_y), self.links.data_ptr(),
                                  self.work.data_ptr(), wb)

    @property
    def volume(self):
        nx, ny, nz, nt = self.n
        return nx * ny * nz * nt

    @property
    def dtype(self):
        return torch.float32 if self.prec == SU2_F32 else torch.float64

    def ref(self):
        return ctypes.byref(self.desc)


def _on_gpu(lat):
    """The library's kernels address device memory: refuse a lattice whose
    storage is not on a GPU before any call reaches them."""
    if not lat.links.is_cuda:
        raise ValueError(f"lattice storage must be on a GPU, not {lat.links.device}")
    return lat


def _tensor(t, lat, dtype, numel, name):
    """Check a caller's output (or input) tensor before its address reaches
    the library: on the lattice's device, of the given dtype, contiguous and
    holding at least numel elements.  Returns t."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device != lat.links.device:
        raise ValueError(f"{name} must be on {lat.links.device}, not {t.device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, not {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name} must hold at least {numel} elements, not {t.numel()}")
    return t


def _rmax(lat):
    return max(1, min(lat.n[:3]) // 2)


def su2_init_cold(lat, stream=None):
    _check(lib.su2_init_cold(_on_gpu(lat).ref(), _stream(stream)))


def su2_init_hot(lat, seed, stream=None):
    _check(lib.su2_init_hot(_on_gpu(lat).ref(), int(seed), _stream(stream)))


def su2_heatbath_sweep(lat, beta, seed, sweep, stream=None):
    _check(lib.su2_heatbath_sweep(_on_gpu(lat).ref(), float(beta), int(seed), int(sweep), _stream(stream)))


def su2_heatbath_halfsweep(lat, beta, seed, sweep, mu, parity, stream=None):
    _check(lib.su2_heatbath_halfsweep(_on_gpu(lat).ref(), float(beta), int(seed), int(sweep), int(mu), int(parity),
                                      _stream(stream)))


def su2_overrelax(lat, n_sweeps=1, stream=None):
    _check(lib.su2_overrelax(_on_gpu(lat).ref(), int(n_sweeps), _stream(stream)))


def su2_overrelax_halfsweep(lat, mu, parity, stream=None):
    _check(lib.su2_overrelax_halfsweep(_on_gpu(lat).ref(), int(mu), int(parity), _stream(stream)))


def su2_plaquette(lat, out=None, stream=None):
    """Enqueue the mean plaquette; returns the device tensor (7 float64):
    [mean, planes 01, 02, 03, 12, 13, 23]."""
    if out is None:
        out = torch.empty(7, dtype=torch.float64, device=lat.device)
    _tensor(out, lat, torch.float64, 7, "out")
    _check(lib.su2_plaquette(_on_gpu(lat).ref(), out.data_ptr(), _stream(stream)))
    return out


def su2_plaquette_noalloc(lat, out, stream=None):
    """su2_plaquette with the library's static scratch in place of the
    lattice's workspace: `out` (7 float64 on the lattice's device) must be
    given, nothing is allocated.  Returns out."""
    _tensor(out, lat, torch.float64, 7, "out")
    _check(lib.su2_plaquette_noalloc(_on_gpu(lat).ref(), out.data_ptr(), _stream(stream)))
    return out


def su2_polyakov(lat, out=None, corr=None, with_corr=True, stream=None):
    """Enqueue the Polyakov loop; returns (out, corr) device tensors:
    out = [mean L, mean |L|], corr = C(r) for r = 1 .. min(Nx,Ny,Nz)/2 (or None)."""
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=lat.device)
    if corr is None and with_corr:
        corr = torch.empty(_rmax(lat), dtype=torch.float64, device=lat.device)
    _tensor(out, lat, torch.float64, 2, "out")
    if corr is not None:
        _tensor(corr, lat, torch.float64, _rmax(lat), "corr")
    _check(lib.su2_polyakov(_on_gpu(lat).ref(), out.data_ptr(), corr.data_ptr() if corr is not None else None,
                            _stream(stream)))
    return out, corr


def su2_heatbath_sweep_measured(lat, beta, seed, sweep, plaq=None, stream=None):
    """Heat-bath sweep that also leaves the plaquette (7 float64, as
    su2_plaquette) of the configuration it produces; returns that tensor."""
    if plaq is None:
        plaq = torch.empty(7, dtype=torch.float64, device=lat.device)
    _tensor(plaq, lat, torch.float64, 7, "plaq")
    _check(lib.su2_heatbath_sweep_measured(_on_gpu(lat).ref(), float(beta), int(seed), int(sweep), plaq.data_ptr(),
                                           _stream(stream)))
    return plaq


def su2_overrelax_measured(lat, n_sweeps=1, plaq=None, stream=None):
    """Overrelaxation sweeps whose last one leaves the plaquette of the final
    configuration; returns that tensor (7 float64)."""
    if plaq is None:
        plaq = torch.empty(7, dtype=torch.float64, device=lat.device)
    _tensor(plaq, lat, torch.float64, 7, "plaq")
    _check(lib.su2_overrelax_measured(_on_gpu(lat).ref(), int(n_sweeps), plaq.data_ptr(), _stream(stream)))
    return plaq


def su2_measure(lat, plaq=None, poly=None, corr=None, with_corr=True, stream=None):
    """Enqueue plaquette and Polyakov loop in one pass; returns (plaq, poly,
    corr) device tensors laid out as su2_plaquette's and su2_polyakov's."""
    if plaq is None:
        plaq = torch.empty(7, dtype=torch.float64, device=lat.device)
    if poly is None:
        poly = torch.empty(2, dtype=torch.float64, device=lat.device)
    if corr is None and with_corr:
        corr = torch.empty(_rmax(lat), dtype=torch.float64, device=lat.device)
    _tensor(plaq, lat, torch.float64, 7, "plaq")
    _tensor(poly, lat, torch.float64, 2, "poly")
    if corr is not None:
        _tensor(corr, lat, torch.float64, _rmax(lat), "corr")
    _check(lib.su2_measure(_on_gpu(lat).ref(), plaq.data_ptr(), poly.data_ptr(),
                           corr.data_ptr() if corr is not None else None, _stream(stream)))
    return plaq, poly, corr


def su2_get_flags(lat, out=None, stream=None):
    if out is None:
        out = torch.empty(1, dtype=torch.int32, device=lat.device)
    _tensor(out, lat, torch.int32, 1, "out")
    _check(lib.su2_get_flags(_on_gpu(lat).ref(), out.data_ptr(), _stream(stream)))
    return out


def su2_batch_table_bytes(count):
    return int(lib.su2_batch_table_bytes(int(count)))


def su2_batch_fill(lattices, betas):
    """Fill and return the host batch table (bytes) for these lattices and betas."""
    count = len(lattices)
    descs = (su2_lattice_t * count)(*[lat.desc for lat in lattices])
    bvals = (ctypes.c_double * count)(*[float(b) for b in betas])
    nbytes = su2_batch_table_bytes(count)
    if nbytes == 0:
        raise Su2Error(SU2_EINVAL, "count must be in [1, 4096]")
    host = (ctypes.c_char * nbytes)()
    _check(lib.su2_batch_fill(descs, bvals, count, host, nbytes))
    return bytes(host), descs


def _batch_on_gpu(batch):
    for lat in batch.lattices:
        _on_gpu(lat)
    if batch.table.device != batch.lattices[0].links.device:
        raise ValueError("the batch table must be on the lattices' device")


class Batch:
    """Independent lattices of one precision updated together: the host table
    filled by su2_batch_fill, copied to a device tensor, plus the host array
    of descriptors the batched calls take."""

    def __init__(self, lattices, betas):
        self.lattices = list(lattices)
        count = len(self.lattices)
        if count != len(betas):
            raise ValueError("one beta per lattice")
        self.count = count
        host, self.descs = su2_batch_fill(self.lattices, betas)
        self.table = torch.frombuffer(bytearray(host), dtype=torch.uint8).to(self.lattices[0].device)
        # the persistent sweep's barrier counter (bits 0-30 zero before and
        # after every call; bit 31 is the barrier phase)
        self.sync = torch.zeros(1, dtype=torch.int32, device=self.lattices[0].links.device)


def su2_batch_heatbath_sweep(batch, seed, sweep=0, d_sweep=None, stream=None):
    """One heat-bath sweep of every lattice; the sweep index is d_sweep[0]
    (a device int32 tensor, read when the kernels run) if given, else sweep."""
    _batch_on_gpu(batch)
    if d_sweep is not None:
        _tensor(d_sweep, batch.lattices[0], torch.int32, 1, "d_sweep")
    _check(lib.su2_batch_heatbath_sweep(batch.descs, batch.count, batch.table.data_ptr(), int(seed), int(sweep),
                                        d_sweep.data_ptr() if d_sweep is not None else None, _stream(stream)))


def su2_batch_overrelax(batch, n_sweeps=1, stream=None):
    _batch_on_gpu(batch)
    _check(lib.su2_batch_overrelax(batch.descs, batch.count, batch.table.data_ptr(), int(n_sweeps),
                                   _stream(stream)))


def su2_batch_sweep(batch, seed, sweep=0, d_sweep=None, n_or=4, spin_limit=0, stream=None):
    """One heat-bath sweep and n_or overrelaxation sweeps of every lattice in
    one persistent launch (bitwise su2_batch_heatbath_sweep followed by
    su2_batch_overrelax(n_or)); the barrier counter is batch.sync."""
    _batch_on_gpu(batch)
    if d_sweep is not None:
        _tensor(d_sweep, batch.lattices[0], torch.int32, 1, "d_sweep")
    _tensor(batch.sync, batch.lattices[0], torch.int32, 1, "batch.sync")
    if not 0 <= int(spin_limit) < (1 << 32):
        raise ValueError("spin_limit must be in [0, 2^32)")
    _check(lib.su2_batch_sweep(batch.descs, batch.count, batch.table.data_ptr(), int(seed), int(sweep),
                               d_sweep.data_ptr() if d_sweep is not None else None, int(n_or),
                               batch.sync.data_ptr(), int(spin_limit), _stream(stream)))


def su2_batch_polyakov(batch, poly=None, corr=None, with_corr=True, stream=None):
    """Polyakov loop (and correlator) of every lattice of the batch, bitwise
    as su2_polyakov of each.  Returns (poly [count, 2] float64, corr
    [count, stride] float64 or None); row j of corr holds C(r), r = 1..
    min(Nx,Ny,Nz)/2 of lattice j, and is left untouched beyond."""
    dev = batch.lattices[0].links.device
    rmax = max(min(lat.n[:3]) // 2 for lat in batch.lattices)
    stride = rmax
    if poly is None:
        poly = torch.empty((batch.count, 2), dtype=torch.float64, device=dev)
    if with_corr and corr is None:
        corr = torch.zeros((batch.count, stride), dtype=torch.float64, device=dev)
    if poly.shape != (batch.count, 2) or poly.dtype != torch.float64 or not poly.is_contiguous():
        raise ValueError("poly must be a contiguous float64 tensor of shape (count, 2)")
    if corr is not None:
        if (corr.dim() != 2 or corr.shape[0] != batch.count or corr.shape[1] < rmax or corr.dtype != torch.float64
                or corr.stride(1) != 1):
            raise ValueError("corr must be a float64 tensor of shape (count, >= max min(Nx,Ny,Nz)/2) with unit "
                             "column stride")
        stride = corr.stride(0)
    if poly.device != dev or (corr is not None and corr.device != dev):
        raise ValueError(f"poly and corr must be on {dev}")
    _batch_on_gpu(batch)
    _check(lib.su2_batch_polyakov(batch.descs, batch.count, batch.table.data_ptr(), poly.data_ptr(),
                                  corr.data_ptr() if corr is not None else None, int(stride), _stream(stream)))
    return poly, corr


def su2_sweep_advance(d_sweep, stream=None):
    """d_sweep[0] += 1 on the device."""
    if not isinstance(d_sweep, torch.Tensor) or not d_sweep.is_cuda or d_sweep.dtype != torch.int32 \
            or d_sweep.numel() < 1:
        raise ValueError("d_sweep must be an int32 tensor on a GPU with at least one element")
    _check(lib.su2_sweep_advance(d_sweep.data_ptr(), _stream(stream)))


# ---------------------------------------------------------------------------
# Learned block proposal
# ---------------------------------------------------------------------------
def su2_lp_param_count():
    return int(lib.su2_lp_param_count())


def su2_lp_workspace_bytes(n):
    return int(lib.su2_lp_workspace_bytes(_dims(n)[1]))


class LPWork:
    """Device workspace of the proposal network for lattices of extents n."""

    def __init__(self, n, device="cuda"):
        nb = su2_lp_workspace_bytes(n)
        if nb == 0:
            raise Su2Error(SU2_EDIMS, "the learned proposal needs Nx, Ny, Nz multiples of 8")
        self.n = tuple(int(v) for v in n)
        self.buf = torch.empty(nb, dtype=torch.uint8, device=device)


def _lp_inputs(lat, params, lpwork):
    _tensor(params, lat, torch.float32, su2_lp_param_count(), "params")
    if lpwork.buf.device != lat.links.device or lpwork.n != lat.n:
        raise ValueError("lpwork must be made for this lattice's extents, on its device")


def su2_lp_forward(lat, params, lpwork, y=None, stream=None):
    """Network outputs y[site*6 + d] (device float32) for the current links."""
    if y is None:
        y = torch.empty(lat.volume * 6, dtype=torch.float32, device=lat.device)
    _lp_inputs(lat, params, lpwork)
    _tensor(y, lat, torch.float32, lat.volume * 6, "y")
    _check(lib.su2_lp_forward(_on_gpu(lat).ref(), params.data_ptr(), lpwork.buf.data_ptr(), lpwork.buf.numel(),
                              y.data_ptr(), _stream(stream)))
    return y


def su2_lp_loss_grad(lat, beta, params, lpwork, grad=None, loss=None, stream=None):
    if grad is None:
        grad = torch.empty(su2_lp_param_count(), dtype=torch.float32, device=lat.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=lat.device)
    _lp_inputs(lat, params, lpwork)
    _tensor(grad, lat, torch.float32, su2_lp_param_count(), "grad")
    _tensor(loss, lat, torch.float64, 1, "loss")
    _check(lib.su2_lp_loss_grad(_on_gpu(lat).ref(), float(beta), params.data_ptr(), lpwork.buf.data_ptr(),
                                lpwork.buf.numel(), grad.data_ptr(), loss.data_ptr(), _stream(stream)))
    return grad, loss


def su2_lp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    for name, t in (("params", params), ("grad", grad), ("m", m), ("v", v)):
        if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.device != params.device
                or t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != params.numel()):
            raise ValueError(f"{name} must be a contiguous float32 tensor on params' GPU with params.numel() "
                             "elements")
    _check(lib.su2_lp_adam(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), params.numel(),
                           int(step), float(lr), float(beta1), float(beta2), float(eps), _stream(stream)))


def su2_lp_move(lat, beta, seed, step, parity, colour, y, accepted, stream=None):
    _tensor(y, lat, torch.float32, lat.volume * 6, "y")
    _tensor(accepted, lat, torch.int32, 1, "accepted")
    _check(lib.su2_lp_move(_on_gpu(lat).ref(), float(beta), int(seed), int(step), int(parity), int(colour), y.data_ptr(),
                           accepted.data_ptr(), _stream(stream)))


def su2_lp_sweep(lat, beta, seed, step, y, accepted, stream=None):
    """All 16 block classes with network outputs y; accepted[0] += accepted moves."""
    _tensor(y, lat, torch.float32, lat.volume * 6, "y")
    _tensor(accepted, lat, torch.int32, 1, "accepted")
    _check(lib.su2_lp_sweep(_on_gpu(lat).ref(), float(beta), int(seed), int(step), y.data_ptr(), accepted.data_ptr(),
                            _stream(stream)))


# ---------------------------------------------------------------------------
# Layout conversion between the library's checkerboard planes and the
# canonical site-major layout U[t][z][y][x][mu][4] (float64, host).  The link
# layout is part of the ABI (include/su2.h); these helpers only re-index.
# ---------------------------------------------------------------------------
def _site_tables(n, device):
    nx, ny, nz, nt = n
    t, z, y, x = torch.meshgrid(*[torch.arange(v, device=device) for v in (nt, nz, ny, nx)], indexing="ij")
    par = ((x + y + z + t) % 2).reshape(-1)
    cb = ((x + nx * (y + ny * (z + nz * t))) // 2).reshape(-1)
    return par, cb


def _planes(lat):
    # (sub-)planes `stride` elements apart; the elements past V/2 are skew
    half = lat.volume // 2
    if lat.prec == SU2_F32:
        stride = int(lib.su2_plane_stride(_dims(lat.n)[1], SU2_F32))
        return lat.links.view(torch.float32).view(4, 2, stride, 4)[:, :, :half]
    stride = int(lib.su2_plane_stride(_dims(lat.n)[1], SU2_F64))
    return lat.links.view(torch.float64).view(4, 2, 2, stride, 2)[:, :, :, :half]


def to_canonical(lat):
    """Copy the links out as a float64 CPU tensor of shape (Nt,Nz,Ny,Nx,4,4)."""
    par, cb = _site_tables(lat.n, lat.device)
    P = _planes(lat)
    if lat.prec == SU2_F32:
        q = P[:, par, cb, :].permute(1, 0, 2)               # (V, mu, 4)
    else:
        q = P[:, par, :, cb, :].reshape(-1, 4, 4)           # (V, mu, sub, 2) -> (V, mu, 4)
    nx, ny, nz, nt = lat.n
    return q.to(torch.float64).cpu().reshape(nt, nz, ny, nx, 4, 4).contiguous()


def from_canonical(lat, U):
    """Overwrite the links from a canonical (Nt,Nz,Ny,Nx,4,4) array (rounded to F32 if needed)."""
    U = torch.as_tensor(U, dtype=torch.float64).reshape(-1, 4, 4).to(lat.device)
    par, cb = _site_tables(lat.n, lat.device)
    P = _planes(lat)
    if lat.prec == SU2_F32:
        P[:, par, cb, :] = U.permute(1, 0, 2).to(torch.float32)
    else:
        P[:, par, :, cb, :] = U.reshape(-1, 4, 2, 2)
