"""The C-ABI library loads and exports what include/fusedir.h declares, and
the Python binding's structs match the C layout.  No GPU calls."""
import ctypes
import json
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fusedir.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(fd_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_function():
    from paper_2604_05794_amd import native
    L = native.lib()
    names = _declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(native.EXPORTS)


def test_struct_layouts_match_the_header():
    from paper_2604_05794_amd import native
    code = r"""
#include <stdio.h>
#include <stddef.h>
#include "fusedir.h"
#define F(s, f) printf("\"%s.%s\": %zu,\n", #s, #f, offsetof(s, f))
int main(void) {
  printf("{\n");
  F(fd_params, width); F(fd_params, refine_step0); F(fd_params, z_near); F(fd_params, mlp);
  F(fd_params, fallback_cost); F(fd_params, proposal_dirs); F(fd_params, head_centre);
  F(fd_params, stream); F(fd_params, ctx);
  F(fd_scene, n_points); F(fd_scene, orient_maps); F(fd_scene, costs); F(fd_scene, head_centre);
  F(fd_camera, R); F(fd_camera, t);
  printf("\"sizeof.fd_params\": %zu, \"sizeof.fd_scene\": %zu, \"sizeof.fd_camera\": %zu,"
         " \"sizeof.fd_adam\": %zu}\n", sizeof(fd_params), sizeof(fd_scene),
         sizeof(fd_camera), sizeof(fd_adam));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        open(c, "w").write(code)
        exe = os.path.join(d, "l")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        lay = json.loads(subprocess.run([exe], capture_output=True, text=True,
                                        check=True).stdout)
    for f in ("width", "refine_step0", "z_near", "mlp", "fallback_cost", "proposal_dirs",
              "head_centre", "stream", "ctx"):
        assert getattr(native.Params, f).offset == lay[f"fd_params.{f}"], f
    for f in ("n_points", "orient_maps", "costs", "head_centre"):
        assert getattr(native.Scene, f).offset == lay[f"fd_scene.{f}"], f
    assert ctypes.sizeof(native.Params) == lay["sizeof.fd_params"]
    assert ctypes.sizeof(native.Scene) == lay["sizeof.fd_scene"]
    assert ctypes.sizeof(native.Adam) == lay["sizeof.fd_adam"]
    assert lay["sizeof.fd_camera"] == 64 and lay["fd_camera.R"] == 16 and lay["fd_camera.t"] == 52


def test_new_struct_layouts_match_the_header():
    from paper_2604_05794_amd import native
    code = r"""
#include <stdio.h>
#include <stddef.h>
#include "fusedir.h"
#define F(s, f) printf("\"%s.%s\": %zu,\n", #s, #f, offsetof(s, f))
int main(void) {
  printf("{\n");
  F(fd_gabor_params, n_orient); F(fd_gabor_params, wavelength); F(fd_gabor_params, out_dtype);
  F(fd_gabor_params, stream); F(fd_gabor_params, ctx);
  F(fd_volume_grid, origin); F(fd_volume_grid, voxel); F(fd_volume_grid, dims);
  F(fd_grow_params, step); F(fd_grow_params, voxel_cap); F(fd_grow_params, seed_mode);
  F(fd_grow_params, centre); F(fd_grow_params, stream); F(fd_grow_params, ctx);
  printf("\"sizeof.fd_gabor_params\": %zu, \"sizeof.fd_volume_grid\": %zu,"
         " \"sizeof.fd_grow_params\": %zu}\n", sizeof(fd_gabor_params),
         sizeof(fd_volume_grid), sizeof(fd_grow_params));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        open(c, "w").write(code)
        exe = os.path.join(d, "l")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        lay = json.loads(subprocess.run([exe], capture_output=True, text=True,
                                        check=True).stdout)
    for cls, cname, fields in (
            (native.GaborParams, "fd_gabor_params",
             ("n_orient", "wavelength", "out_dtype", "stream", "ctx")),
            (native.VolumeGrid, "fd_volume_grid", ("origin", "voxel", "dims")),
            (native.GrowParams, "fd_grow_params",
             ("step", "voxel_cap", "seed_mode", "centre", "stream", "ctx"))):
        for f in fields:
            assert getattr(cls, f).offset == lay[f"{cname}.{f}"], (cname, f)
        assert ctypes.sizeof(cls) == lay[f"sizeof.{cname}"], cname


def test_defaults_follow_the_paper():
    from paper_2604_05794_amd import native
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_hyperparameters.json")))
    p = native.Params()
    native.lib().fd_params_init(ctypes.byref(p))
    assert p.top_k == g["top_k"] and p.patch == g["patch"]
    assert p.mode == native.FD_MODE_PLAIN and p.map_dtype == native.FD_F16


def test_error_string_is_thread_local_and_empty_initially():
    from paper_2604_05794_amd import native
    assert native.lib().fd_last_error() is not None


def test_product_path_does_not_reach_the_oracle():
    """The package and its native library never name the oracle."""
    pkg = os.path.join(ROOT, "paper_2604_05794_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "fdo_" not in txt and "liboracle" not in txt, f
