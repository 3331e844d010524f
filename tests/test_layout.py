"""The front end's parameter layouts (CPU): the C-ABI keeps geometry
component-major and moves the colour arrays Gaussian-major; the conversion
round-trips and puts each Gaussian's colour coefficients side by side."""
import numpy as np

from paper_2501_00342_amd import raster, scenes


def test_colour_is_gaussian_major_and_round_trips():
    sc, _ = scenes.small_clustered(37, 5, 32, 32)
    dev = {k: raster.to_device_layout(k, getattr(sc, k)) for k in scenes.FIELDS}
    n, nc, K = sc.n, (sc.sh_degree + 1) ** 2, sc.n_lobes
    assert dev["means"].shape == (3, n) and dev["opacity_logits"].shape == (n,)
    assert dev["sh"].shape == (n, nc, 3) and dev["sg_axes"].shape == (n, K, 3)
    assert dev["sg_log_sharpness"].shape == (n, K) and dev["sg_amplitudes"].shape == (n, K, 3)
    g = 11
    # Gaussian g's SH block is one contiguous run of 3 (L+1)^2 floats
    flat = dev["sh"].reshape(-1)
    assert np.array_equal(flat[g * 3 * nc:(g + 1) * 3 * nc], sc.sh[:, :, g].reshape(-1))
    assert np.array_equal(dev["sg_amplitudes"].reshape(-1)[g * 3 * K:(g + 1) * 3 * K],
                          sc.sg_amplitudes[:, :, g].reshape(-1))
    back = raster.to_scene_layout(dev)
    for k in scenes.FIELDS:
        assert back[k].shape == getattr(sc, k).shape and np.array_equal(back[k], getattr(sc, k)), k


def test_packed_colour_records_are_views_of_one_buffer():
    import torch
    sc, _ = scenes.small_clustered(29, 6, 32, 32)
    p = raster.params_to_device(sc, "cpu", packed=True)
    rs = raster.colour_record_floats(sc.sh_degree, sc.n_lobes)
    assert raster.colour_stride(p) == rs
    base = p["sh"].data_ptr()
    nc3 = 3 * (sc.sh_degree + 1) ** 2
    for k, off in (("sh", 0), ("sg_axes", nc3), ("sg_log_sharpness", nc3 + 3 * sc.n_lobes),
                   ("sg_amplitudes", nc3 + 4 * sc.n_lobes)):
        assert p[k].data_ptr() == base + 4 * off and p[k].stride(0) == rs, k
        assert np.array_equal(p[k].numpy(), raster.to_device_layout(k, getattr(sc, k))), k
    flat = raster.params_to_device(sc, "cpu", packed=False)
    assert raster.colour_stride(flat) == 0
    g = raster.new_grads(p)
    assert all(t.is_contiguous() and t.shape == p[k].shape for k, t in g.items())
    assert isinstance(g["sh"], torch.Tensor)
