"""The resolution schedule's host code (gs_resolution_schedule and
gs_schedule_resolution, no GPU) against the FP64 oracle (Sec. 4.2, Eq. 2;
supplementary Eq. 6-7), on frequency maps the oracle computes."""
import numpy as np
import pytest

from oracle import schedule as O
from paper_2503_18402_amd import gsmi


@pytest.fixture(scope="module")
def L():
    if not gsmi.is_available():
        from paper_2503_18402_amd import build
        build.build()
    return gsmi.lib()


@pytest.mark.parametrize("norm", ["sum", "mean"])
@pytest.mark.parametrize("shape,m,a", [((2, 3, 64, 96), 4, 4.0), ((1, 3, 133, 200), 6, 4.0),
                                       ((3, 3, 45, 61), 3, 2.5)])
def test_knots_match_oracle(L, shape, m, a, norm):
    rng = np.random.default_rng(sum(shape))
    imgs = rng.uniform(size=shape)
    imgs += np.linspace(0, 1, shape[-1])[None, None, None, :]   # some low-frequency content
    Mc = O.magnitude_map(imgs)                                   # centred
    r_o, s_o, _ = O.schedule_knots(Mc, 6000, a=a, m=m, norm=norm)
    r_c, s_c = gsmi.gs_resolution_schedule(np.fft.ifftshift(Mc), 6000, a=a, m=m, norm=norm)
    assert np.allclose(r_c, r_o, rtol=1e-12, atol=0)
    assert np.allclose(s_c, s_o, rtol=1e-12, atol=1e-9)
    for k in np.linspace(0, 6500, 57):
        assert gsmi.gs_schedule_resolution(k, r_c, s_c) == pytest.approx(
            O.resolution_at(k, r_o, s_o), rel=1e-12)


def test_schedule_argument_errors(L):
    m = np.ones((8, 8))
    with pytest.raises(gsmi.GsError):
        gsmi.gs_resolution_schedule(m, 100, a=1.0)
    with pytest.raises(gsmi.GsError):
        gsmi.gs_resolution_schedule(m, 0)
    with pytest.raises(gsmi.GsError):
        gsmi.gs_resolution_schedule(m, 100, m=0)
    assert L.gs_frequency_map(1, 5000, 10, 256, 256, 256, 1 << 30, None) == 1
    assert L.gs_frequency_map(0, 10, 10, 256, 256, 256, 1 << 30, None) == 1
    assert L.gs_frequency_map(1, 10, 10, 256, 256, 256, 16, None) == 2
    assert L.gs_downsample_aa(1, 10, 10, 0, 5, 256, 256, None) == 1
    assert gsmi.gs_frequency_map_workspace_bytes(4097, 10) == 0
