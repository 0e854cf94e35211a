"""GPU tests of the C ABI's caller buffers: fields and states read into, or
written from, host memory (pageable numpy arrays, pinned torch tensors) equal
bit for bit what device buffers give, and host memory is refused where the
state itself must live (lbm_create's dev_buf)."""
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


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_host_buffers_equal_device_buffers(prec):
    """A ragged 20x14x11 cavity at an odd and an even time: fields and state
    through numpy host arrays are bit for bit those through device tensors;
    set_state from host arrays gives the same lattice as from device tensors."""
    wl = lbm_inputs.cavity((20, 14, 11), seed=21)
    _say(f"case host buffers {prec} 20x14x11")
    with Lattice(wl, prec, check_interval=10) as lat:
        for steps in (7, 6):
            lat.step(steps)
            dev = {k: v.cpu().numpy() for k, v in lat.fields().items()}
            host = lat.fields(host=True)
            for k in FIELDS:
                assert np.array_equal(dev[k], host[k]), (lat.time, k)
            fd, gd = lat.get_state()
            fh, gh = lat.get_state(host=True)
            assert np.array_equal(fd.cpu().numpy(), fh) and np.array_equal(gd.cpu().numpy(), gh), lat.time
        # perturb, set from host arrays and from device tensors, compare the next steps
        rng = np.random.default_rng(7)
        f1 = fh * (1.0 + 1e-3 * rng.standard_normal(fh.shape))
        g1 = gh + 1e-3 * rng.standard_normal(gh.shape)
        with Lattice(wl, prec) as other:
            # the same time counter: FP16 storage draws its rounding bits from it
            other.step(lat.time)
            lat.set_state(f1, g1)                                    # numpy: host memory
            other.set_state(torch.from_numpy(f1).cuda(), torch.from_numpy(g1).cuda())
            a_f, a_g = lat.get_state(host=True)
            b_f, b_g = other.get_state(host=True)
            assert np.array_equal(a_f, b_f) and np.array_equal(a_g, b_g)
            lat.step(3)
            other.step(3)
            a = lat.fields(host=True)
            b = other.fields(host=True)
            for k in FIELDS:
                assert np.array_equal(a[k], b[k]), k


def test_pinned_host_memory_and_null_outputs():
    """Pinned host memory (torch pin_memory) and a NULL output through the C
    ABI directly: the written fields equal the device ones, the skipped one is
    untouched."""
    wl = lbm_inputs.cavity((16, 12, 10), seed=3)
    _say("case pinned host memory 16x12x10 fp64")
    lib = lbm.library()
    with Lattice(wl, "fp64") as lat:
        lat.step(5)
        ref = {k: v.cpu().numpy() for k, v in lat.fields().items()}
        out = {k: torch.full(lat.shape, -7.0, dtype=torch.float64, pin_memory=True) for k in FIELDS}
        ptrs = [ctypes.c_void_p(out[k].data_ptr()) if k != "uy" else None for k in FIELDS]
        assert lib.lbm_fields(lat._h, *ptrs) == 0
        for k in FIELDS:
            if k == "uy":
                assert bool((out[k] == -7.0).all())
            else:
                assert np.array_equal(out[k].numpy(), ref[k]), k


def test_create_refuses_host_memory_as_the_state_buffer():
    """lbm_create with dev_buf in host memory (a numpy buffer, a pinned
    tensor) returns LBM_ERR_INVALID_ARG and creates nothing."""
    wl = lbm_inputs.cavity(8)
    p = lbm.make_params(wl, "fp32")
    need = lbm.required_bytes(p)
    lib = lbm.library()
    _say("case create with host dev_buf")
    host = np.zeros(need + 256, dtype=np.uint8)
    base = (host.ctypes.data + 255) // 256 * 256
    h = ctypes.c_void_p()
    st = lib.lbm_create(ctypes.byref(p), ctypes.c_void_p(base), ctypes.c_size_t(need), None, ctypes.byref(h))
    assert st == 1 and not h.value, (st, lib.lbm_last_error())
    assert b"host memory" in lib.lbm_last_error()
    pinned = torch.zeros(need + 256, dtype=torch.uint8, pin_memory=True)
    base = (pinned.data_ptr() + 255) // 256 * 256
    st = lib.lbm_create(ctypes.byref(p), ctypes.c_void_p(base), ctypes.c_size_t(need), None, ctypes.byref(h))
    assert st == 1 and not h.value
    # the library is still usable afterwards (no error left behind)
    with Lattice(wl, "fp32") as lat:
        lat.step(2)
        assert lat.time == 2


def test_nusselt_start_collects_the_state_it_started_on():
    """lbm_nusselt_start enqueues the reduction of the current state; the next
    lbm_nusselt collects it even when steps were enqueued in between, and the
    call after that reduces the state of its own time."""
    wl = lbm_inputs.cavity((20, 16, 12), porosity=0.5, darcy=1e-2, rayleigh=5e3, seed=23)
    print("case nusselt_start fp32 20x16x12", flush=True)
    with Lattice(wl, "fp32") as lat:
        lat.step(40)
        ref = lat.nusselt()
        lat.nusselt_start()
        lat.step(7)
        assert lat.nusselt() == ref
        now = lat.nusselt()
        assert now != ref and now[0] != 0.0
        lat.nusselt_start()
        assert lat.nusselt() == now
        # a reduction started on one stream and collected after a stream change
        lat.step(5)
        later = lat.nusselt()
        lat.nusselt_start()
        other = torch.cuda.Stream()
        assert lbm.library().lbm_set_stream(lat._h, ctypes.c_void_p(other.cuda_stream)) == 0
        lat.stream = other
        assert lat.nusselt() == later
