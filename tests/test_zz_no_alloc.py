"""The allocation-free FFT entry point (pm_fft_noalloc) against the entry point it varies (pm_debug_fft,
whose scratch is the context's spectrum buffer) through the C ABI: two calls in a row on one GPU, the
second on a smaller mesh, forward and inverse, in both precisions, at the FFT parity bars of the path
(FP32 1e-5, FP64 1e-10 relative L2; the two share their kernels, so the outputs agree far closer).  A
mesh whose padded spectrum does not fit the fixed scratch array is refused with PM_ERANGE."""
import numpy as np
import pytest

from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BAR = {"fp32": 1e-5, "fp64": 1e-10}


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_fft_noalloc_matches_debug_fft(precision):
    from paper_2607_17929_amd import PMContext, PMError
    from paper_2607_17929_amd import _lib as L
    from paper_2607_17929_amd.pm import fft_noalloc
    print(f"fft without allocation, {precision}", flush=True)
    lib = L.load()
    assert lib.pm_fft_noalloc_scratch_bytes(128, L.PM_FP64) <= L.PM_FFT_NOALLOC_SCRATCH_BYTES
    for n, seed in ((64, 1), (32, 2)):  # the second call on a smaller mesh
        r = np.random.default_rng(seed)
        f = torch.tensor(r.standard_normal((n, n, n)), device="cuda")
        ctx = PMContext(n, 8, 100.0, physics="newtonian", precision=precision)
        ref_k = ctx.debug_fft(f, 1)
        got_k = fft_noalloc(f, n, 1, precision)
        torch.cuda.synchronize()
        ek = max(rel_l2(got_k.real.cpu().numpy(), ref_k.real.cpu().numpy()),
                 rel_l2(got_k.imag.cpu().numpy(), ref_k.imag.cpu().numpy()))
        ref_x = ctx.debug_fft(ref_k, -1)
        got_x = fft_noalloc(ref_k, n, -1, precision)
        torch.cuda.synchronize()
        ex = rel_l2(got_x.cpu().numpy(), ref_x.cpu().numpy())
        print(f"  n = {n}: forward {ek:.1e}, inverse {ex:.1e} (bitwise equal: "
              f"{bool(torch.equal(got_k, ref_k))}, {bool(torch.equal(got_x, ref_x))})", flush=True)
        assert ek < BAR[precision] and ex < BAR[precision]
        del ctx
    big = 256 if precision == "fp32" else 256
    x = torch.zeros((big, big, big), device="cuda")
    with pytest.raises(PMError) as e:
        fft_noalloc(x, big, 1, precision)
    assert e.value.status == L.PM_ERANGE
