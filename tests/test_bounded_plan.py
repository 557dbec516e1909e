"""Plans with a bounded workspace (sfft_analyze_bounded, host only): the
levels are formed by list scheduling within the bound, so the workspace
stays within it while the circuit (its netlist hash and products) is the
same; a bound no schedule meets is refused.  The plaintext evaluation of
bounded schedules against the netlist runs in the sanitizer host check;
their ciphertexts are compared with the unbounded plan's on the GPU."""
import pytest

from paper_1611_08769_amd import sfft as S


def _shape_params(dims, L, F, f, cplx, n):
    shp = S.shape(dims, L, F, f, cplx)
    return shp, S.sfft_size_params(shp, n)


@pytest.mark.parametrize("geo", [(2, 8, 8, 4, False, 1), (1, 32, 12, 6, True, 1)])
def test_bounded_workspace_fits(geo):
    shp, p = _shape_params(*geo)
    free = S.sfft_analyze(shp, p)
    for frac in (0.7, 0.5, 0.35):
        lim = int(free.ws_bytes * frac)
        b = S.sfft_analyze_bounded(shp, p, lim)
        assert b.ws_bytes <= lim
        assert b.exec_products == free.exec_products and b.products == free.products
        assert bytes(b.netlist_sha256) == bytes(free.netlist_sha256)
        assert b.levels >= free.levels
        assert b.exec_steps == b.levels + 2


def test_unbounded_is_the_default_plan():
    shp, p = _shape_params(1, 16, 8, 4, True, 1)
    a, b = S.sfft_analyze(shp, p), S.sfft_analyze_bounded(shp, p, 0)
    assert (a.levels, a.ws_bytes, a.ws_cts) == (b.levels, b.ws_bytes, b.ws_cts)


def test_bound_too_small_is_refused():
    shp, p = _shape_params(1, 8, 8, 4, False, 1)
    with pytest.raises(S.SfftError) as ei:
        S.sfft_analyze_bounded(shp, p, S.sfft_ct_bytes(p))
    assert ei.value.code == S.SFFT_ENOMEM
    with pytest.raises(S.SfftError) as ei:
        S.sfft_analyze_bounded(shp, p, -1)
    assert ei.value.code == S.SFFT_EINVAL
