"""The allocation-free loss entry point against the workspace one (GPU).

gp_l1_dssim_loss_grad_noalloc keeps its scratch in a static device array shared
by every call on the GPU.  Two calls in a row, the second on a smaller batch
(so that stale contents of the first are left in the array), must give the
gradient and the loss terms of gp_l1_dssim_loss_grad bit for bit; a batch
beyond the array's capacity is refused before anything is launched.
"""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

from paper_2603_20611_amd import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[no-alloc] {msg}", flush=True)
    sys.stdout.flush()


def _pair(n_slices, width, height, seed):
    rng = np.random.default_rng(seed)
    img = rng.uniform(0.0, 1.0, (n_slices, height, width)).astype(np.float32)
    tgt = (img * synth.speckle(img.shape, seed + 1)).astype(np.float32)
    tgt[:, ::7, ::5] = img[:, ::7, ::5]          # ties of the L1 term
    return torch.from_numpy(img.ravel()).cuda(), torch.from_numpy(tgt.ravel()).cuda()


def _both(img, tgt, n_slices, width, height, ws):
    from paper_2603_20611_amd import render
    g_ws = torch.full_like(img, 7.0)
    l_ws = torch.zeros(2, device="cuda")
    render.l1_dssim_loss_grad(img, tgt, n_slices, width, height, ws, lam=0.2, grad=g_ws, loss=l_ws)
    g_na = torch.full_like(img, -3.0)
    l_na = torch.zeros(2, device="cuda")
    render.l1_dssim_loss_grad_noalloc(img, tgt, n_slices, width, height, lam=0.2, grad=g_na, loss=l_na)
    torch.cuda.synchronize()
    return g_ws, l_ws, g_na, l_na


def test_noalloc_loss_matches_workspace_loss(gp):
    from paper_2603_20611_amd import render
    ws = render.Workspace()
    # the training batch of the benchmark (8 slices of 256 x 256), then a smaller,
    # ragged one (3 slices of 100 x 70)
    for n_slices, width, height, seed in ((8, 256, 256, 1), (3, 100, 70, 2)):
        _say(f"{n_slices} slices of {width} x {height}")
        img, tgt = _pair(n_slices, width, height, seed)
        g_ws, l_ws, g_na, l_na = _both(img, tgt, n_slices, width, height, ws)
        assert torch.equal(g_na, g_ws), "gradient differs from the workspace entry point"
        assert torch.equal(l_na, l_ws), "loss terms differ from the workspace entry point"
        assert float(l_ws[1]) > 0.0


def test_noalloc_loss_refuses_too_large(gp):
    from paper_2603_20611_amd import binding as B
    lib = B.load()
    img = torch.zeros(1, device="cuda")
    # 9 slices of 512 x 512: 2,359,296 pixels, beyond the static scratch
    st = lib.gp_l1_dssim_loss_grad_noalloc(C.c_void_p(img.data_ptr()), C.c_void_p(img.data_ptr()), 9, 512, 512,
                                           C.c_float(0.2), C.c_void_p(img.data_ptr()), None, None)
    assert st == B.GP_EINVAL
    assert b"static scratch" in lib.gp_last_error()
