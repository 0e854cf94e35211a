"""Host-side behaviour of bench.py that needs no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_the_traffic_profile_names_the_kernel_it_was_taken_on():
    """The counter summary the bench line reads carries the hash of the
    kernel sources it was measured on, and a byte count per launch of the
    right size (the 208 B/node algorithmic bytes, within a few per cent)."""
    with open(os.path.join(ROOT, "profiles", "step_cavity256_fp32_traffic.json")) as f:
        rec = json.load(f)
    assert len(rec["kernel_hash"]) == 16 and int(rec["kernel_hash"], 16) >= 0
    algorithmic = 208 * rec["nodes"]
    assert 1.0 <= rec["bytes_per_launch"] / algorithmic < 1.05


def test_the_valu_profile_names_the_kernel_it_was_taken_on():
    """The FP16-mode instruction counts the bench line reads carry the same
    kernel hash as the traffic profile and lie between the static counts of
    the two parities' kernels' lean paths (about 600 to 1200 per wavefront)."""
    with open(os.path.join(ROOT, "profiles", "step_cavity256_fp32_traffic.json")) as f:
        traffic = json.load(f)
    for stem in ("step_cavity256_fp16", "step_channel512x128x128_fp16"):
        with open(os.path.join(ROOT, "profiles", f"{stem}_valu.json")) as f:
            rec = json.load(f)
        assert rec["kernel_hash"] == traffic["kernel_hash"]
        waves = rec["nodes"] // 64
        assert 600 <= rec["even_valu"] / waves < rec["odd_valu"] / waves <= 1200
        assert rec["valu_per_step"] == (rec["even_valu"] + rec["odd_valu"]) / 2


def test_the_kernel_hash_ignores_comments_and_sees_code():
    """The source hash that ties profiles to kernels drops C++ and Python
    comments and blank lines, and nothing else."""
    sys.path.insert(0, ROOT)
    import bench
    cpp = "int a = 1;  // one\n\n/* block\n comment */ int b = 2;\n"
    assert bench._code_of("x.hpp", cpp) == bench._code_of("x.hpp", "int a = 1;\n int b = 2;")
    assert bench._code_of("x.hpp", cpp) != bench._code_of("x.hpp", cpp.replace("2;", "3;"))
    py = "FLAGS = ['-O3']  # optimise\n# note\n"
    assert bench._code_of("b.py", py) == "FLAGS = ['-O3']"
    assert bench._code_of("b.py", py) != bench._code_of("b.py", py.replace("-O3", "-O2"))
