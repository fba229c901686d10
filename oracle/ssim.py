"""FP64 reference of the slice loss L = L1 + lambda * D-SSIM and its gradient.

TEST INFRASTRUCTURE ONLY: imported by the test-suite alone.  Shares no code
with the HIP path.

The paper's loss (Sec. 4.3, loss function; lambda = 0.2 in Sec. 5.1) adds a
D-SSIM term to L1.  SSIM is the structural similarity of Wang et al. 2004
(cited by the paper for its metrics):
  S(p) = (2 mu_x mu_y + C1)(2 sigma_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2))
with local statistics taken under an 11 x 11 Gaussian window of standard
deviation 1.5 (normalised to unit sum), C1 = (0.01 L)^2, C2 = (0.03 L)^2.
Readings taken where the paper is silent: dynamic range L = 1; the window
sees zeros outside the slice ("same"-size output); D-SSIM = 1 - the mean of
S over every pixel of the batch; L1 = the mean of |I - T| over the batch.
The gradient is the float64 automatic derivative of this definition.
"""
import numpy as np
import torch
import torch.nn.functional as F

F64 = torch.float64
WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window():
    """The 11 x 11 Gaussian window (sigma 1.5), unit sum, float64 [11, 11]."""
    k = torch.arange(WINDOW, dtype=F64) - (WINDOW // 2)
    g = torch.exp(-(k * k) / (2.0 * SIGMA * SIGMA))
    g = g / g.sum()
    return torch.outer(g, g)


def _filter(img):
    """Window-weighted local sums of img [S, H, W] with zeros outside."""
    w = window()[None, None]
    return F.conv2d(img[:, None], w, padding=WINDOW // 2)[:, 0]


def ssim_map(x, y):
    """SSIM at every pixel of x, y [S, H, W] (float64 tensors)."""
    mx, my = _filter(x), _filter(y)
    sxx = _filter(x * x) - mx * mx
    syy = _filter(y * y) - my * my
    sxy = _filter(x * y) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def loss(image, target, lam=0.2):
    """(L, L1, D-SSIM, dL/dimage) for image, target [S, H, W]; values float, gradient numpy float64."""
    x = torch.as_tensor(np.asarray(image), dtype=F64).clone().requires_grad_(True)
    y = torch.as_tensor(np.asarray(target), dtype=F64)
    l1 = (x - y).abs().mean()
    dssim = 1.0 - ssim_map(x, y).mean()
    total = l1 + lam * dssim
    total.backward()
    return float(total.detach()), float(l1.detach()), float(dssim.detach()), x.grad.numpy()
