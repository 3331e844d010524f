"""GPU parity of the fused Adam step (render_adam_step) against the FP64
oracle's Adam with the staged SG start, over several iterations on both
sides of sg_start, for interleaved and separate colour arrays and the
orthogonal lobe forms."""
import numpy as np
import pytest
import torch

from oracle import optim as O
from paper_2501_00342_amd import optim, raster, scenes

pytestmark = pytest.mark.gpu

FIELDS = scenes.FIELDS


def _host(d):
    return raster.to_scene_layout({k: v.detach().cpu().numpy().astype(np.float64)
                                   for k, v in d.items()})


@pytest.mark.parametrize("form,packed", [("sg", True), ("sg", False), ("world", True),
                                         ("frame", True)])
def test_adam_matches_oracle_across_sg_start(form, packed):
    n = 3001
    if form == "sg":
        sc = scenes.clustered_scene(n, 5, 1, 4, n_clusters=10)
    else:
        mode = scenes.LOBES_WORLD if form == "world" else scenes.LOBES_FRAME
        sc = scenes.orthogonal_scene(n, 5, mode, 2, n_clusters=10)
    cam = scenes.config1_camera(64, 48)
    rast = raster.Rasterizer.for_scene(sc, [cam], scenes.Options())
    params = raster.params_to_device(sc, packed=packed)
    assert (raster.colour_stride(params) > 0) == packed
    lr = dict(optim.DEFAULT_LR)
    opt = optim.Adam(rast, params, lr=lr, sg_start=3)
    P = _host(params)
    M = {k: np.zeros_like(a) for k, a in P.items()}
    V = {k: np.zeros_like(a) for k, a in P.items()}
    rng = np.random.default_rng(9)
    for step in range(1, 6):
        G = {k: rng.normal(0.0, 1e-3, size=a.shape).astype(np.float32) for k, a in P.items()}
        gdev = {k: torch.from_numpy(np.ascontiguousarray(raster.to_device_layout(k, G[k]))).cuda()
                for k in FIELDS}
        opt.step(gdev)
        P, M, V = O.adam_step(P, {k: g.astype(np.float64) for k, g in G.items()}, M, V, lr, step,
                              sg_start=3)
        torch.cuda.synchronize()
        got_p, got_m, got_v = _host(params), _host(opt.exp_avg), _host(opt.exp_avg_sq)
        for k in FIELDS:
            if P[k].size == 0:
                continue
            scale = np.abs(P[k]).max() + 1e-30
            assert np.abs(got_p[k] - P[k]).max() <= 2e-6 * scale, (form, step, k)
            # m = b1 m + (1 - b1) g in float32 can cancel: the floor is a few
            # float32 roundings of the array's largest moment (over 5 steps)
            m_floor = 1e-6 * np.abs(M[k]).max()
            assert np.all(np.abs(got_m[k] - M[k]) <= 1e-5 * np.abs(M[k]) + m_floor), (form, step, k)
            assert np.allclose(got_v[k], V[k], rtol=1e-5, atol=1e-15), (form, step, k)
            if k in O.LOBE_FIELDS and step < 3:
                assert not got_m[k].any(), (form, step, k)


def test_adam_leaves_padding_of_interleaved_records_alone():
    """The update writes only the colour floats of each record, not the
    padding that rounds a record to 16 bytes."""
    sc = scenes.orthogonal_scene(1000, 6, scenes.LOBES_FRAME, 2, n_clusters=5)
    cam = scenes.config1_camera(64, 48)
    rast = raster.Rasterizer.for_scene(sc, [cam], scenes.Options())
    params = raster.params_to_device(sc, packed=True)
    base = params["sh"]
    stride = base.stride(0)
    rs = raster.colour_record_floats(sc.sh_degree, sc.n_lobes, sc.lobe_mode)
    assert stride > rs
    buf = torch.as_strided(base, (sc.n, stride), (stride, 1))
    buf[:, rs:] = 7.0
    opt = optim.Adam(rast, params, sg_start=0)
    grads = {k: torch.ones(tuple(v.shape), dtype=torch.float32, device=v.device)
             for k, v in params.items()}
    opt.step(grads)
    torch.cuda.synchronize()
    assert bool((buf[:, rs:] == 7.0).all())
