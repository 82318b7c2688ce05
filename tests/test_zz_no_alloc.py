"""nic_psnr_noalloc, the entry point that allocates nothing (its per-block partial sums live in a
static device array of the library), against nic_psnr (partials in the model's workspace) and an
FP64 host evaluation, through the C ABI: two calls in a row, the second with a smaller input
(fewer blocks than the first left in the shared array), plus the degenerate and refused cases."""
import ctypes as C
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2506_19742_amd import nic, synth  # noqa: E402

pytestmark = pytest.mark.gpu

MAX_N = 4096 * 65536


def _noalloc(gt, pred, n=None):
    out = C.c_double(-1.0)
    st = nic.lib().nic_psnr_noalloc(C.c_void_p(gt.data_ptr()), C.c_void_p(pred.data_ptr()),
                                    gt.numel() if n is None else n,
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(out))
    return st, out.value


def test_noalloc_psnr_matches_psnr():
    w = synth.WORKLOADS["tiny64"]
    print("[case] nic_psnr_noalloc: model for nic_psnr", flush=True)
    m = nic.Model(nic.config_for(w), synth.cone_geometry(w.n_det, w.n_views))
    rng = np.random.default_rng(5)
    try:
        for n in (3_000_001, 70_000):
            print(f"[case] nic_psnr_noalloc n={n}", flush=True)
            a = (rng.random(n) * 0.05).astype(np.float32)
            b = (a + rng.standard_normal(n) * 1e-3).astype(np.float32)
            gt, pred = torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda")
            st, got = _noalloc(gt, pred)
            assert st == 0, nic.lib().nic_last_error().decode()
            ref = m.psnr(gt, pred)
            a64, b64 = a.astype(np.float64), b.astype(np.float64)
            host = 10.0 * math.log10(a64.max() ** 2 / np.mean((b64 - a64) ** 2))
            assert abs(got - ref) <= 1e-12 * abs(ref)
            assert abs(got - host) <= 1e-9 * abs(host)
        st, v = _noalloc(gt, gt)
        assert st == 0 and v == math.inf
        for bad in (0, -1, MAX_N + 1):     # refused before any launch
            st, _ = _noalloc(gt, pred, n=bad)
            assert st == nic.NIC_EINVAL
            assert "n" in nic.lib().nic_last_error().decode()
    finally:
        m.close()
