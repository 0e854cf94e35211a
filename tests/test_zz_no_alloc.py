"""GPU test of lbm_fields_noalloc, the entry point for callers that cannot
allocate: through the C ABI, its output equals lbm_fields' bit for bit, on two
calls in a row, the second on a smaller lattice.  The first lattice needs
three passes through the library's 16 MiB staging array (ragged last pass);
outputs mix pageable host memory, pinned host memory, device memory and NULL."""
import ctypes
import sys

import numpy as np
import pytest

import lbm_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_1611_03329_amd import Lattice, lbm  # noqa: E402

FIELDS = ("rho", "ux", "uy", "uz", "T")
SCRATCH_BYTES = 16 << 20


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _noalloc(lat, kinds):
    """lbm_fields_noalloc into buffers of the given kinds ('host', 'pinned',
    'device' or None per field); returns host copies (None where skipped)."""
    bufs = {}
    for k, kind in zip(FIELDS, kinds):
        if kind == "host":
            bufs[k] = np.full(lat.shape, np.nan)
        elif kind == "pinned":
            bufs[k] = torch.full(lat.shape, float("nan"), dtype=torch.float64, pin_memory=True)
        elif kind == "device":
            bufs[k] = torch.full(lat.shape, float("nan"), dtype=torch.float64, device=lat.device)
        else:
            bufs[k] = None

    def ptr(b):
        if b is None:
            return None
        return ctypes.c_void_p(b.ctypes.data if isinstance(b, np.ndarray) else b.data_ptr())

    st = lbm.library().lbm_fields_noalloc(lat._h, *(ptr(bufs[k]) for k in FIELDS))
    assert st == 0, lbm.library().lbm_last_error()
    torch.cuda.synchronize()
    out = {}
    for k, b in bufs.items():
        if b is None:
            out[k] = None
        elif isinstance(b, np.ndarray):
            out[k] = b
        else:
            out[k] = b.cpu().numpy()
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_fields_equal_lbm_fields(prec):
    big = lbm_inputs.cavity((120, 100, 80), seed=11)     # 960,000 nodes: 3 passes with 5 host outputs
    small = lbm_inputs.cavity((20, 14, 11), seed=12)
    assert 2 * SCRATCH_BYTES // (8 * 5) < 120 * 100 * 80 < 3 * SCRATCH_BYTES // (8 * 5)
    cases = [(big, 9, ("host", "host", "host", "host", "host")),
             (small, 4, ("host", "pinned", None, "device", "host"))]
    for wl, steps, kinds in cases:
        _say(f"case noalloc {prec} {wl['nx']}x{wl['ny']}x{wl['nz']} after {steps} steps, outputs {kinds}")
        with Lattice(wl, prec) as lat:
            lat.step(steps)
            ref = {k: v.cpu().numpy() for k, v in lat.fields().items()}
            got = _noalloc(lat, kinds)
            for k in FIELDS:
                if got[k] is None:
                    continue
                assert np.array_equal(got[k], ref[k]), (prec, wl["nx"], k)
