"""Learned frames through the C ABI: the coarse render plus the upsampler when
the validation passes, the plain render when it does not, decided on the
device."""
import numpy as np
import pytest

from oracle import cnn
from paper_1205_0282_amd import binding, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    vol = synth.make_cube(synth.RECIPE_SMALL, workers=4)
    vmin, vmax = float(vol.min()), float(vol.max())
    rgba = synth.ramp_tf(vmin, vmax)
    dims = vol.shape[::-1]
    views = [synth.orbit_view(dims, f, kind="persp", width=160, height=120) for f in (3, 30)]
    coarse_views = [synth.orbit_view(dims, f, kind="persp", width=80, height=60, step=2.0) for f in (3, 30)]

    def caster(n_views, w, h):
        bc = binding.BrickCaster(0)
        bc.plan(dims, (64, 64, 64), max_views=n_views, max_w=w, max_h=h)
        bc.bind()
        bc.load(torch.from_numpy(vol).cuda())
        bc.set_transfer_function(rgba, vmin, vmax)
        return bc

    learned = caster(2, 160, 120)
    learned.cnn_setup(2, 60, 80)
    params = cnn.init_params(21)
    learned.cnn_set_weights(params)
    plain = caster(2, 160, 120)
    yield dict(vol=vol, views=views, coarse_views=coarse_views, learned=learned, plain=plain, caster=caster)
    learned.close()
    plain.close()


def test_learned_frame_is_upsampled_coarse_render(setup):
    import torch
    L, P = setup["learned"], setup["plain"]
    L.set_learned(True, coarse_step=2.0, psnr_threshold_db=-1e9, validate_stride=4)
    L.set_views(setup["views"])
    out = L.render().clone()
    st = L.stats()
    assert st["fell_back"] == 0 and np.isfinite(st["psnr_db"])
    # the same coarse render and upsampling through the separate entry points
    C = setup["caster"](2, 80, 60)
    C.set_views(setup["coarse_views"])
    coarse = C.render()
    up = L.cnn_forward(coarse)
    torch.cuda.synchronize()
    assert torch.equal(out, up)
    C.close()


def test_learned_frame_falls_back_to_plain(setup):
    import torch
    L, P = setup["learned"], setup["plain"]
    L.set_learned(True, coarse_step=2.0, psnr_threshold_db=1e9, validate_stride=8)
    L.set_views(setup["views"])
    out = L.render().clone()
    st = L.stats()
    assert st["fell_back"] == 1
    P.set_views(setup["views"])
    ref = P.render()
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    # plain frames report no validation
    L.set_learned(False)
    L.render()
    st = L.stats()
    assert st["fell_back"] == -1 and np.isnan(st["psnr_db"])


def test_validation_psnr_matches_host(setup):
    """With stride 1 every tile is validated: the reported PSNR is the PSNR of
    the whole upsampled frame against the plain frame."""
    import torch
    L, P = setup["learned"], setup["plain"]
    L.set_learned(True, coarse_step=2.0, psnr_threshold_db=-1e9, validate_stride=1)
    L.set_views(setup["views"])
    out = L.render().cpu().numpy().astype(np.float64)
    st = L.stats()
    P.set_views(setup["views"])
    ref = P.render().cpu().numpy().astype(np.float64)
    mse = np.mean((out - ref) ** 2)
    assert abs(st["psnr_db"] - 10 * np.log10(1 / mse)) < 1e-3


def test_concurrent_validation_pass_measures_the_same_frame(setup):
    """With stride 2 the validation pass runs on the second stream beside the
    coarse pass and the network.  Its PSNR must be the PSNR over one tile of
    every 2x2 block of tiles of the upsampled frame against the plain frame:
    it lies between the best and the worst of the four possible selections,
    and repeated frames give the same images."""
    import torch
    L, P = setup["learned"], setup["plain"]
    L.set_learned(True, coarse_step=2.0, psnr_threshold_db=-1e9, validate_stride=2)
    L.set_views(setup["views"])
    P.set_views(setup["views"])
    ref = P.render().cpu().numpy().astype(np.float64)
    first = None
    for _ in range(3):
        out = L.render().cpu().numpy().astype(np.float64)
        st = L.stats()
        if first is None:
            first = out
        assert np.array_equal(out, first)
        err = (out - ref) ** 2
        psnrs = []
        for oy in range(2):
            for ox in range(2):
                sel = np.zeros(out.shape[1:3], bool)
                for ty in range(oy, (out.shape[1] + 7) // 8, 2):
                    for tx in range(ox, (out.shape[2] + 7) // 8, 2):
                        sel[ty * 8:ty * 8 + 8, tx * 8:tx * 8 + 8] = True
                psnrs.append(10 * np.log10(1 / err[:, sel].mean()))
        assert min(psnrs) - 1e-3 <= st["psnr_db"] <= max(psnrs) + 1e-3
        assert any(abs(st["psnr_db"] - p) < 1e-3 for p in psnrs)
