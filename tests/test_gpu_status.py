"""The on-device status paths (GPU): a pair count past the workspace's
capacity in the unchecked (graph) mode, and device cameras that disagree
with the host cameras.  Both are bounded paths: the kernels clamp every
write to the workspace and set a status bit."""
import numpy as np
import pytest
import torch

from oracle import forward as F
from paper_2501_00342_amd import _lib as L
from paper_2501_00342_amd import raster, scenes
from tests import parity
from tests.gpu_util import camera_numpy

pytestmark = pytest.mark.gpu

CANARY = 0xA5


def _with_canary(rast, extra=1 << 16):
    """Put the rasteriser's workspace at the start of a larger buffer whose
    tail holds a known byte pattern."""
    nbytes = rast.ws.numel()
    big = torch.full((nbytes + extra,), CANARY, dtype=torch.uint8, device=rast.device)
    rast.ws = big[:nbytes]
    return big, nbytes


def test_unchecked_capacity_overflow_truncates_within_the_workspace():
    sc, cam = scenes.small_clustered(4000, 41, 120, 80)
    opts = scenes.Options()
    pre = F.preprocess(sc, cam, opts)
    keys, vals, nt = F.emit_pairs(pre)
    P = int(keys.size)
    assert P > 2000
    cap = P // 3
    rast = raster.Rasterizer.for_scene(sc, [cam], opts, capacity=cap, auto_grow=False)
    big, nbytes = _with_canary(rast)
    params = raster.params_to_device(sc)
    out = rast.new_outputs()
    rast.forward(params, out=out, check=False)
    torch.cuda.synchronize()
    bits, pairs = rast.status()
    assert bits & L.SGS_STATUS_CAPACITY
    assert pairs == P
    tail = big[nbytes:].cpu().numpy()
    assert (tail == CANARY).all(), "bytes past the workspace were written"
    # the checked mode reports the overflow instead of rendering ...
    with pytest.raises(L.SgsError):
        rast.forward(params, check=True)
    # ... and with growth allowed renders the oracle's image
    rast.auto_grow = True
    out = rast.forward(params, check=True)
    bits, pairs = rast.status()
    assert bits == 0 and pairs == P and rast.capacity >= P
    img, dep, T, n = camera_numpy(out, [cam])
    rep = parity.compare_image(img, dep, T, n, F.render(sc, cam, opts))
    assert rep["bad"] == 0, rep


@pytest.mark.parametrize("what", ["width", "znear"])
def test_device_camera_mismatch_sets_status_and_writes_no_image(what):
    sc, cam = scenes.small_clustered(2000, 42, 64, 48)
    opts = scenes.Options()
    rast = raster.Rasterizer.for_scene(sc, [cam], opts)
    params = raster.params_to_device(sc)
    good = rast.forward(params, check=True).image.clone()
    raw = rast.dev_cams.cpu().numpy().copy()
    if what == "width":
        raw[0:4] = np.frombuffer(np.int32(cam.width + 16).tobytes(), np.uint8)
    else:
        off = 4 * (2 + 9 + 3 + 4)     # znear
        raw[off:off + 4] = np.frombuffer(np.float32(-1.0).tobytes(), np.uint8)
    rast.dev_cams = torch.from_numpy(raw).to(rast.device)
    out = rast.new_outputs()
    for t in (out.image, out.final_T):
        t.fill_(-3.0)
    rast.forward(params, out=out, check=False)
    torch.cuda.synchronize()
    bits, _ = rast.status()
    assert bits & L.SGS_STATUS_CAMERAS
    assert bool((out.image == -3.0).all()) and bool((out.final_T == -3.0).all())
    # the checked forward reports it as an error
    with pytest.raises(L.SgsError):
        rast.forward(params, check=True)
    # restoring the cameras restores the image
    rast.dev_cams = torch.frombuffer(bytearray(bytes(rast.host_cams)), dtype=torch.uint8).to(rast.device)
    assert torch.equal(rast.forward(params, check=True).image, good)
