"""Host-side logic that needs no GPU: serving pool sizing."""
import pytest

from paper_1812_01502_amd.serving import CTL_BYTES, PARAM_BYTES, slot_footprint, slots_for_budget


def test_control_and_parameter_sizes_match_the_device_structs():
    """The footprint constants equal sizeof(Ctl) and sizeof(ModelParams<float>)."""
    import os
    import shutil
    import subprocess
    import tempfile
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = (
        "#define __device__\n#define __host__\n#define __forceinline__ inline\n"
        "#include <cstdint>\n#include <cstdio>\n"
        f'#include "{root}/include/pf.h"\n'
        "namespace pfk { constexpr int kMaxDim = PF_MAX_DIM; }\n"
    )
    # the two structs are plain data: compile their definitions out of pf_device.h
    dev = open(os.path.join(root, "paper_1812_01502_amd", "csrc", "pf_device.h")).read()
    import re
    mp = re.search(r"template <typename T> struct ModelParams \{.*?\n\};", dev, re.S).group(0)
    consts = "\n".join(re.findall(r"constexpr int k(?:Off\w+|MaxPending) = [^;]+;", dev))
    ctl = re.search(r"struct Ctl \{.*?\n\};", dev, re.S).group(0)
    src += "namespace pfk {\n" + consts + "\n" + mp + "\n" + ctl + "\n}\n"
    src += 'int main(){printf("%zu %zu\\n", sizeof(pfk::Ctl), sizeof(pfk::ModelParams<float>));}\n'
    d = tempfile.mkdtemp()
    try:
        open(os.path.join(d, "s.cpp"), "w").write(src)
        subprocess.run([cxx, "-std=c++17", os.path.join(d, "s.cpp"), "-o", os.path.join(d, "s")], check=True)
        out = subprocess.run([os.path.join(d, "s")], capture_output=True, text=True, check=True).stdout.split()
    finally:
        shutil.rmtree(d, ignore_errors=True)
    assert (int(out[0]), int(out[1])) == (CTL_BYTES, PARAM_BYTES)


def test_slot_footprint_counts_every_buffer():
    # states (2 buffers x d planes) + log-weights (2 buffers) + partial records
    # + control block + model parameters + record
    assert slot_footprint(1, 4096) == 2 * 4096 * 4 + 2 * 4096 * 4 + 8 * 7 * 4 + CTL_BYTES + PARAM_BYTES + 304
    assert slot_footprint(16, 1 << 20) > slot_footprint(4, 1 << 20) > slot_footprint(1, 1 << 20)


@pytest.mark.parametrize("budget", [1 << 26, 1 << 30, 24 << 30])
def test_slots_for_budget_fits(budget):
    dims = {"sv": 1, "lg4": 4}
    shapes = {("sv", 4096): 1.0, ("lg4", 1 << 16): 1.0, ("lg4", 1 << 20): 2.0}
    cnt = slots_for_budget(shapes, dims, budget)
    used = sum(slot_footprint(dims[m], n) * c for (m, n), c in cnt.items())
    assert all(c >= 1 for c in cnt.values())
    # each pool stays within its share (pools of one slot may exceed a tiny budget)
    for (m, n), c in cnt.items():
        share = budget * shapes[(m, n)] / sum(shapes.values())
        assert c == 1 or c * slot_footprint(dims[m], n) <= share
    assert used <= budget or min(cnt.values()) == 1
