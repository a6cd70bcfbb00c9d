import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def c4_net():
    """The post-process trained on the GPU by the library's own kernels: 1800
    hemisphere views of the 50M-point vector field at 512 x 512 (the 9:1
    training split of 2000), splat targets with sigma 1.5 px, 2500 Adam steps
    of batch 16.  Yields the scene, the weights, 16 training views' inputs
    (FP8 calibration) and the 200 held-out cameras."""
    import time
    torch = pytest.importorskip("torch")
    from paper_2407_19097_amd import scenes, train
    log = lambda m: print(f"  [c4] {m}", flush=True)
    print("\n[fixture] training the post-process: 1800 views of the vector field at 512x512, 2500 steps", flush=True)
    t0 = time.time()
    sc = scenes.vector_field(device="cuda")
    w, cal, heldout, secs, losses = train.train_c4(sc, log=log)
    log(f"done in {time.time() - t0:.0f} s (training {secs:.0f} s)")
    yield {"scene": sc, "weights": w, "cal": cal, "heldout": heldout, "losses": losses}
    w.close()
    del sc, cal
    torch.cuda.empty_cache()
