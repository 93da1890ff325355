"""su2_plaquette_noalloc: the plaquette without a workspace, its partials in
the library's static device array, called through the C ABI with a
descriptor that has no workspace, against su2_plaquette on the same links.
Both run the same kernels in the same order, so the results must be
bitwise equal.  Two calls in a row, the second on a smaller lattice (the
array keeps the first call's partials; nothing may leak into the second)."""
import ctypes

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def su2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1104_5432_amd as m
    return m


def _noalloc(su2, lat, out):
    # the descriptor without a workspace, straight through the C ABI
    d = su2.su2_lattice_t((ctypes.c_int32 * 4)(*lat.n), lat.prec, lat.desc.lattice_id, lat.desc.tile,
                          lat.desc.tile_y, lat.links.data_ptr(), None, 0)
    rc = su2.lib.su2_plaquette_noalloc(ctypes.byref(d), out.data_ptr(),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == su2.SU2_OK, su2.lib.su2_last_error()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_plaquette_equals_plaquette(su2, prec):
    shapes = [(64, 64, 64, 64), (6, 4, 10, 8)]      # the second smaller (and with a ragged last block)
    walks = [(8, 8), (0, 0)]
    for k, (n, (tile, tile_y)) in enumerate(zip(shapes, walks)):
        print(f"no-alloc plaquette {n} {prec}, call {k + 1}", flush=True)
        lat = su2.Lattice(n, prec, device="cuda", tile=tile, tile_y=tile_y)
        su2.su2_init_hot(lat, 1234 + k)
        su2.su2_heatbath_sweep(lat, 2.3, 1234 + k, 0)
        ref = su2.su2_plaquette(lat)
        got = torch.full((7,), -1.0, dtype=torch.float64, device="cuda")
        _noalloc(su2, lat, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (n, (got - ref).abs().max().item())
        assert 0.0 < got[0].item() < 1.0
        del lat
    # the binding under the same name
    lat = su2.Lattice((8, 8, 8, 4), prec, device="cuda")
    su2.su2_init_hot(lat, 7)
    out = torch.empty(7, dtype=torch.float64, device="cuda")
    su2.su2_plaquette_noalloc(lat, out)
    ref = su2.su2_plaquette(lat)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
