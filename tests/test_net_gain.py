"""What the trained network gains over the method without it.

The post-process is trained on the GPU by the library's own forward and
backward kernels (400 hemisphere views of the 50M-point vector field at
512 x 512, splat targets with sigma 1.5 px, 9:1 split, Adam lr 1e-3, batch
16) and evaluated on the 40 held-out views.  The baseline is the
rasterizer's RGB G-buffer alone (points as pixels), the analogue of the
paper's CR row.  Pass: the network is at least 3 dB better and reaches
30 dB PSNR against the splat."""
import math

import pytest

from paper_2407_19097_amd import narvis, scenes, train

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_trained_network_beats_raster_rgb():
    print("\n[case] train 150 steps on 360 views, evaluate 40 held-out views", flush=True)
    sc = scenes.vector_field(device="cuda")
    r = train.Renderer(sc, 512, 512)
    cams = train.hemisphere_views(400, (0.5, 0.5, 0.2), 0.75 * math.sqrt(2.16), seed=4)
    feats, targets = train.render_dataset(r, cams, log=lambda m: print(m, flush=True))
    w = narvis.NetWeights(train.init_blob(0))
    losses, _ = train.train(w, feats[:360], targets[:360], 150, batch=16, log=lambda m: print(m, flush=True))
    p_net, p_ras, s_net, s_ras = train.evaluate(w, feats[360:], targets[360:])
    print(f"  PSNR net {p_net:.2f} dB vs raster RGB {p_ras:.2f} dB; SSIM {s_net:.3f} vs {s_ras:.3f}", flush=True)
    w.close()
    assert losses[-1][1] < losses[0][1]
    assert p_net >= p_ras + 3.0
    assert p_net >= 30.0
