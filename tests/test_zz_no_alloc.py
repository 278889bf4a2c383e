"""The no-allocation entry point fcd_deformation_noalloc (GPU, through the C ABI) against
fcd_deformation on the same phase planes: bit-for-bit equal, on two calls in a row, the
second on a smaller lattice, in FP64 and FP32; sizes beyond its array are rejected."""
import sys

import numpy as np
import pytest

from fcd_inputs import single_channel_small

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("no GPU", allow_module_level=True)

from paper_2410_11129_amd import fcd  # noqa: E402
from paper_2410_11129_amd.sim import Channel  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def noalloc(ch):
    out = torch.full((4,), float("nan"), dtype=torch.float64, device=ch.device)
    fcd.fcd_deformation_noalloc(ch.lat, ch.phi.data_ptr(), ch.stream.cuda_stream, out.data_ptr())
    ch.stream.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("precision", [fcd.FCD_FP64, fcd.FCD_FP32])
def test_noalloc_deformation_equals_handle_deformation(precision):
    big = single_channel_small().replace(nx=640, ny=160, xc=200.0, yc=79.5, r_core=20.0, r_shell=40.0)
    small = single_channel_small()  # 200 x 50
    for w in (big, small):  # the second call on a smaller lattice reuses the array
        say(f"case noalloc deformation {w.nx}x{w.ny} precision {precision}")
        ch = Channel(w, precision=precision)
        ch.init_droplet()
        ch.step(30)
        want = np.array(ch.deformation())  # refreshes the phase planes, then reduces
        got = noalloc(ch)
        assert np.array_equal(got, want), (got, want)
        assert got[2] > 0 and got[3] > 0
        ch.close()


def test_noalloc_rejects_sizes_beyond_its_array():
    import ctypes as C
    lat = fcd.fcd_lattice(8, fcd.FCD_NOALLOC_MAX_NY + 2, fcd.FCD_FP64, 8)
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    st = fcd.lib().fcd_deformation_noalloc(C.byref(lat), C.c_void_p(out.data_ptr()), None, C.c_void_p(out.data_ptr()))
    assert st == fcd.FCD_ERR_ARG and "FCD_NOALLOC_MAX_NY" in fcd.fcd_last_error()
