"""ptflash_flash_noalloc (the flash with the library's own static device
scratch as its workspace) against ptflash_flash with a caller's workspace,
through the C ABI: bit-identical outputs on two calls in a row, the second
with a smaller input (the scratch keeps the first call's contents, which
must not leak into the second).  The size limit is checked on the CPU
(tests/test_capi.py)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2205_03090_amd import _capi, api, workloads  # noqa: E402
from parity import gpu_to_numpy  # noqa: E402

pytestmark = pytest.mark.gpu

KEYS = ("label", "beta", "x", "y", "iters", "status", "flops", "tm")


def _both(w, **kw):
    a = api.flash(w.z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij, **kw)
    b = api.flash(w.z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij, noalloc=True, **kw)
    torch.cuda.synchronize()
    return gpu_to_numpy(a), gpu_to_numpy(b)


@pytest.mark.parametrize("nc,n1,n2,form", [(8, 60_000, 7_001, _capi.FORM_PERSISTENT),
                                           (20, 20_000, 3_333, _capi.FORM_PERSISTENT),
                                           (8, 20_000, 5_555, _capi.FORM_PLAIN)])
def test_noalloc_equals_flash_on_two_calls(nc, n1, n2, form):
    print(f"case noalloc nc={nc} n={n1} then {n2}", flush=True)
    base = workloads.uniform_workload("na", 5100 + nc, n1, nc, 0.5, (200.0, 600.0), (1e5, 2e7))
    for n in (n1, n2):
        w = base.subset(np.arange(n))
        a, b = _both(w, form=form)
        assert (a["label"] == 1).mean() > 0.05
        for k in KEYS:
            ga = a.get(k)
            gb = b.get(k)
            assert ga is not None and np.array_equal(ga, gb, equal_nan=True), (n, k)
