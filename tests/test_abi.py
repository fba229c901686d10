"""The C-ABI library loads and exports every function include/gaussianpile.h declares (CPU only)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gaussianpile.h")
LIB = os.path.join(ROOT, "paper_2603_20611_amd", "libgaussianpile.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gp_render_slices", "gp_render_backward", "gp_adam_step", "gp_l1_loss_grad",
                     "gp_workspace_create", "gp_workspace_destroy", "gp_debug_export_bins"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_loads_and_binding_matches_header():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name)
    from paper_2603_20611_amd import binding
    assert set(binding.exported_names()) <= set(declared_functions())
    lib.gp_version.restype = ctypes.c_int32
    assert lib.gp_version() >= 100


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_side_validation_without_gpu():
    """Argument checks run on the host before any device call."""
    from paper_2603_20611_amd import binding as B
    lib = B.load()
    o = B.RenderOpts()
    assert lib.gp_default_opts(ctypes.byref(o)) == 0
    assert abs(o.q_cut - 11.0825) < 1e-3 and o.bbox_sigmas == 3.0 and o.scale_mod == 1.0
    assert lib.gp_default_opts(None) == B.GP_EINVAL
    cfg = B.AdamCfg((ctypes.c_float * 4)(1, 1, 1, 1), 0.9, 0.999, 1e-15, 0, 0)
    assert lib.gp_adam_step(None, None, None, None, 0, 0, ctypes.byref(cfg), None) == B.GP_EINVAL
    assert b"step" in lib.gp_last_error()
    assert lib.gp_l1_loss_grad(None, None, -1, 1.0, None, None, None) == B.GP_EINVAL
    assert lib.gp_render_slices(None, None, None, 0, None, None, None) == B.GP_EINVAL
    # the allocation-free loss refuses a batch beyond its static scratch before any device call
    fake = ctypes.c_void_p(256)
    assert lib.gp_l1_dssim_loss_grad_noalloc(fake, fake, 9, 512, 512, ctypes.c_float(0.2), fake, None,
                                             None) == B.GP_EINVAL
    assert b"static scratch" in lib.gp_last_error()
    assert lib.gp_l1_dssim_loss_grad_noalloc(fake, fake, -1, 512, 512, ctypes.c_float(0.2), fake, None,
                                             None) == B.GP_EINVAL
