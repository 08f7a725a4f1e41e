"""The README's C example, built against include/raptor.h and the library and run as a plain C
process: it traces its 512 x 512 image at 230 GHz on an all-zero grid (no emission) and reports
the ray-steps, which depend on the geometry alone and so equal those of the same call through
the Python binding."""
import os
import re
import subprocess

import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_c_example_runs(tmp_path):
    from paper_1801_10452_amd import raptor as R
    with open(os.path.join(ROOT, "README.md")) as f:
        src = re.findall(r"```c\n(.*?)```", f.read(), flags=re.S)[0]
    (tmp_path / "app.c").write_text(src)
    lib_dir = os.path.dirname(R.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-O1", str(tmp_path / "app.c"), "-I" + os.path.join(ROOT, "include"),
                    "-L" + lib_dir, "-lraptor_hip", "-Wl,-rpath," + lib_dir, "-o", str(tmp_path / "app")],
                   check=True, timeout=120)
    print("[c example] built; running", flush=True)
    r = subprocess.run([str(tmp_path / "app")], capture_output=True, text=True, timeout=120)
    print(f"[c example] rc={r.returncode} out={r.stdout.strip()} err={r.stderr.strip()[-300:]}", flush=True)
    assert r.returncode == 0
    m = re.match(r"(\S+) Jy, (\d+) ray-steps in (\S+) ms", r.stdout.strip())
    assert m and float(m.group(1)) == 0.0
    ctx = R.Context(0)
    grid = S.constant_grid((0.0, 0.0, 0.0, 0.0), n1=256, n2=256, r_in=1.1, r_out=50.0, hslope=0.3,
                           dtype=np.float32, a_gen=0.9375)
    gh = ctx.upload_grid(grid)
    cam = S.Camera(spin=0.9375, incl_deg=60.0, nx=512, ny=512, r_cam=1e4, fov_half=20.0)
    _, flux, st = ctx.trace_spectrum(cam, gh, [230e9], R.default_opts(transfer_prec=R.F32))
    ctx.release_grid(gh)
    ctx.close()
    assert st.ray_steps == int(m.group(2)) and flux[0] == 0.0
