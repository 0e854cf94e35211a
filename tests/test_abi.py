"""CPU checks of the C ABI: the built library exports every function that
include/lbm.h declares, the ctypes structs match the C layout, and parameter
validation rejects bad input before any device work."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")
LIB = os.path.join(ROOT, "paper_1611_03329_amd", "liblbm.so")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("lbm_create", "lbm_step", "lbm_fields", "lbm_nusselt", "lbm_residual",
                 "lbm_totals", "lbm_destroy", "lbm_required_bytes"):
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(lbm_\w+)", out))
    missing = [n for n in _declared_functions() if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(LIB)
    for n in _declared_functions():
        getattr(lib, n)


def test_ctypes_layout_matches_c_header():
    """Compiles a tiny C program against include/lbm.h and compares sizeof and
    every field offset with the ctypes mirror."""
    from paper_1611_03329_amd import lbm
    fields = [f for f, _ in lbm.Params._fields_]
    prog = ["#include <stdio.h>", "#include <stddef.h>", '#include "lbm.h"', "int main(void){",
            'printf("%zu %zu %zu %zu\\n", sizeof(lbm_params), sizeof(lbm_face), sizeof(lbm_derived), sizeof(lbm_launch));',
            'printf("%zu %zu %zu %zu\\n", offsetof(lbm_launch, block), offsetof(lbm_launch, blocks_per_cu), '
            'offsetof(lbm_launch, group_bytes), offsetof(lbm_launch, xcd_ranges));']
    for f in fields:
        prog.append(f'printf("%zu\\n", offsetof(lbm_params, {f}));')
    prog.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write("\n".join(prog))
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True,
                                               check=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(lbm.Params)
    assert vals[1] == ctypes.sizeof(lbm.Face)
    assert vals[2] == ctypes.sizeof(lbm.Derived)
    assert vals[3] == ctypes.sizeof(lbm.Launch)
    assert vals[4:8] == [getattr(lbm.Launch, f).offset for f, _ in lbm.Launch._fields_]
    for f, off in zip(fields, vals[8:]):
        assert getattr(lbm.Params, f).offset == off, f


def test_validation_rejects_bad_parameters():
    import lbm_inputs
    from paper_1611_03329_amd import lbm
    ok = lbm.make_params(lbm_inputs.cavity(8))
    assert lbm.required_bytes(ok) > 0
    bad = [dict(porosity=0.0), dict(porosity=1.2), dict(darcy=0.0), dict(prandtl=0.0),
           dict(s_nu_set=2.5), dict(zeta_alpha_set=2.0), dict(rayleigh=0.0), dict(nx=0),
           dict(lattice=27), dict(varpi=1.0), dict(gravity_axis=3), dict(init_axis=4)]
    for kw in bad:
        p = lbm.make_params(lbm_inputs.cavity(8, **kw))
        with pytest.raises(lbm.LBMError) as ei:
            lbm.required_bytes(p)
        assert ei.value.status == 1, kw
    # unsupported precision and mismatched periodic faces
    p = lbm.make_params(lbm_inputs.cavity(8), precision=7)
    with pytest.raises(lbm.LBMError) as ei:
        lbm.required_bytes(p)
    assert ei.value.status == 5
    wl = lbm_inputs.cavity(8)
    wl["faces"][0] = lbm_inputs.face("periodic", "periodic")
    with pytest.raises(lbm.LBMError):
        lbm.required_bytes(lbm.make_params(wl))


def test_create_rejects_before_touching_the_device():
    """lbm_create validates first: on a machine without a GPU it still returns
    the validation error, never a device error."""
    import lbm_inputs
    from paper_1611_03329_amd import lbm
    lib = lbm.library()
    p = lbm.make_params(lbm_inputs.cavity(8, porosity=-1.0))
    h = ctypes.c_void_p()
    st = lib.lbm_create(ctypes.byref(p), None, 0, None, ctypes.byref(h))
    assert st == 1 and not h.value
    assert b"porosity" in lib.lbm_last_error()
    # a caller buffer that is too small is refused before any device call
    p = lbm.make_params(lbm_inputs.cavity(8))
    st = lib.lbm_create(ctypes.byref(p), ctypes.c_void_p(256), 16, None, ctypes.byref(h))
    assert st == 2 and not h.value


def test_required_bytes_layout():
    import lbm_inputs
    from paper_1611_03329_amd import lbm
    n = 32 ** 3
    b64 = lbm.required_bytes(lbm.make_params(lbm_inputs.cavity(32), "fp64"))
    b32 = lbm.required_bytes(lbm.make_params(lbm_inputs.cavity(32), "fp32"))
    # one copy of 26 populations plus a 4-field snapshot, in the storage precision
    assert 26 * n * 8 + 4 * n * 8 <= b64 < 26 * n * 8 + 4 * n * 8 + (1 << 20)
    assert 26 * n * 4 + 4 * n * 4 <= b32 < 26 * n * 4 + 4 * n * 4 + (1 << 20)
    b15 = lbm.required_bytes(lbm.make_params(lbm_inputs.cavity(32, lattice=15), "fp32"))
    assert b15 < b32
    # FP16 storage: the 19 flow populations in FP16, the 7 temperature populations in FP32
    b16 = lbm.required_bytes(lbm.make_params(lbm_inputs.cavity(32), "fp16"))
    assert (19 * 2 + 7 * 4) * n + 4 * n * 4 <= b16 < (19 * 2 + 7 * 4) * n + 4 * n * 4 + (1 << 20)


def test_size_limits_are_exact():
    """Byte offsets inside a population region are 32-bit: a region (the moving
    flow populations, (q - 1) planes of the node count rounded up to whole
    tiles of 2048) must stay below 4 GiB, and a box below 2^30 nodes.  The
    largest FP32 D3Q19 box of this shape is accepted, one more z layer is not;
    FP16 storage halves the flow region and takes it."""
    import lbm_inputs
    from paper_1611_03329_amd import lbm
    largest = lbm_inputs.cavity((400, 384, 388))       # 59,596,800 nodes: 18 * 4 B * n < 2^32
    over = lbm_inputs.cavity((400, 384, 389))          # 59,750,400 nodes: 18 * 4 B * n >= 2^32
    assert 18 * 4 * 400 * 384 * 388 < 1 << 32 <= 18 * 4 * 400 * 384 * 389
    assert lbm.required_bytes(lbm.make_params(largest, "fp32")) > 26 * 4 * 400 * 384 * 388
    with pytest.raises(lbm.LBMError) as ei:
        lbm.required_bytes(lbm.make_params(over, "fp32"))
    assert ei.value.status == 5
    assert lbm.required_bytes(lbm.make_params(over, "fp16")) > 0
    with pytest.raises(lbm.LBMError) as ei:
        lbm.required_bytes(lbm.make_params(largest, "fp64"))
    assert ei.value.status == 5
    with pytest.raises(lbm.LBMError) as ei:
        lbm.required_bytes(lbm.make_params(lbm_inputs.cavity((1024, 1024, 1025)), "fp16"))
    assert ei.value.status == 1
