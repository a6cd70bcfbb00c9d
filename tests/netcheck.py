"""Helpers shared by the network tests (no arithmetic of the method: the
forward pass itself is the oracle's)."""
import numpy as np

from oracle import net as onet

# Farther than any output's dependence on the input (about 61 pixels for the
# four-level network: two 3x3 convolutions per level and per decoder stage,
# doubled by each pooling, plus the bilinear taps), and a multiple of 8.
CROP_MARGIN = 96


def crop_forward(P, x, y0, y1, x0, x1, margin=CROP_MARGIN):
    """Oracle forward outputs [:, :, y0:y1, x0:x1] of the full image x, computed
    on a crop that extends `margin` pixels past the tile (clipped at the image
    border).  Tile corners and margin are multiples of 8, so the crop keeps
    the pooling grid of the full image and the tile's outputs are the
    full-image ones."""
    N, C, H, W = x.shape
    assert y0 % 8 == 0 and x0 % 8 == 0 and y1 % 8 == 0 and x1 % 8 == 0 and margin % 8 == 0
    cy0, cy1 = max(0, y0 - margin), min(H, y1 + margin)
    cx0, cx1 = max(0, x0 - margin), min(W, x1 + margin)
    y, _ = onet.forward(P, x[:, :, cy0:cy1, cx0:cx1])
    return y[:, :, y0 - cy0:y1 - cy0, x0 - cx0:x1 - cx0]
