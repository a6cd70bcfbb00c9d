"""The benchmark's command line: one GPU only (a run asking for more exits
with status 2 and says why), and the U-Net FLOP count it reports."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_unet_flop_count_matches_the_oracle_layers():
    """2 x multiply-adds per full-resolution pixel, summed over the layers the
    oracle lists (a level-l layer covers 4^-l of the pixels)."""
    sys.path.insert(0, ROOT)
    import bench
    from oracle import unet as ounet
    for widths in (ounet.WIDTHS, (32, 32, 64, 64, 64)):
        want = 0.0
        for name, kind, shape, _ in ounet.layers(widths):
            if name == "head" or name == "desc":
                level = 0
            elif name.startswith("enc") or name.startswith("dec"):
                level = int(name[3:])
            else:  # up_l runs on the grid of level l + 1
                level = int(name[2:]) + 1
            macs = 1
            for d in shape:
                macs *= d
            want += 2.0 * macs / 4 ** level
        assert abs(bench.unet_flop_per_px(widths) - want) <= 1e-9 * want
