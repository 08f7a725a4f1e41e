"""The C-ABI library loads and exports every entry point declared in include/raptor.h, and the
host-side work counts are available without a GPU."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "raptor.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(raptor_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import ctypes
    from paper_1801_10452_amd import raptor as R
    lib = R.lib()
    names = declared_symbols()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(R.EXPORTS) == sorted(n for n in names if n in R.EXPORTS)
    assert set(names) <= set(R.EXPORTS) | {n for n in names if n.startswith("raptor_mlp")}


def test_struct_sizes_match_header_layout(tmp_path):
    """The binding's ctypes structures have the sizes and field offsets a C compiler gives the
    header's structures."""
    import ctypes
    import subprocess
    from paper_1801_10452_amd import raptor as R
    assert ctypes.sizeof(R.CCamera) == 48
    assert ctypes.sizeof(R.COpts) == 16 + 24 + 40 + 8 + 8 + 8
    assert ctypes.sizeof(R.CGridDesc) == 16 + 48 + 8 + 32 + 8 + 8 + 32
    assert ctypes.sizeof(R.CStats) == 104
    pairs = {"raptor_camera": R.CCamera, "raptor_opts": R.COpts, "raptor_grid_desc": R.CGridDesc,
             "raptor_stats": R.CStats, "raptor_plan": R.CPlan}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "raptor.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{cname}.{f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, py in pairs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert int(got[f"{cname}.{f[0]}"]) == getattr(py, f[0]).offset, (cname, f[0])


def test_work_per_unit_counts():
    from paper_1801_10452_amd import raptor as R
    w = R.work_per_unit()
    # 4 RHS evaluations dominate an RK4 step; 4 sincos + 4 reciprocals + 1 step division
    assert 400 < w["step_flops"] < 1200 and w["step_special"] == 9
    assert w["sample_flops"] > 50 and w["freq_flops"] > 10


def test_no_device_reports_cleanly():
    from paper_1801_10452_amd import raptor as R
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(R.RaptorError) as e:
        R.Context(0)
    assert e.value.status == R.E_DEVICE


def test_work_per_step_of_each_integrator():
    """Connection evaluations per step: RK4 four, RK2 two, Verlet one, corrected Verlet two."""
    from paper_1801_10452_amd import raptor as R
    rk4 = R.work_per_step(R.RK4)
    assert rk4[0] == R.work_per_unit()["step_flops"]
    rk2, ver, vcor = R.work_per_step(R.RK2), R.work_per_step(R.VERLET), R.work_per_step(R.VERLET_CORRECTED)
    assert ver[0] < rk2[0] < rk4[0] and ver[0] < vcor[0] < rk4[0]
    # each connection evaluation takes one reciprocal, each RK stage one sin/cos of theta
    assert rk4[1] - rk2[1] == 4 and vcor[1] - ver[1] == 1
    # one derivative evaluation (plus the corrector's update) is the difference between
    # corrected and plain Verlet; the stage updates add the rest
    per_eval = vcor[0] - ver[0]
    assert rk2[0] == pytest.approx(2 * per_eval, rel=0.25)
    assert rk4[0] == pytest.approx(4 * per_eval, rel=0.25)
    with pytest.raises(R.RaptorError):
        R.work_per_step(7)


def test_readme_c_example_compiles_and_links(tmp_path):
    """The C example of the README compiles against the header with every warning as an error,
    and links against the built library (no GPU is touched: it is not run)."""
    import subprocess
    from paper_1801_10452_amd import raptor as R
    with open(os.path.join(ROOT, "README.md")) as f:
        blocks = re.findall(r"```c\n(.*?)```", f.read(), flags=re.S)
    assert len(blocks) == 1
    src = tmp_path / "app.c"
    src.write_text(blocks[0])
    lib_dir = os.path.dirname(R.LIB_PATH) if hasattr(R, "LIB_PATH") else os.path.join(ROOT, "paper_1801_10452_amd")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", str(src), "-I" + os.path.join(ROOT, "include"),
           "-L" + lib_dir, "-lraptor_hip", "-Wl,--unresolved-symbols=ignore-in-shared-libs", "-o", str(tmp_path / "app")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
