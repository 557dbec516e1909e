"""GPU: the whole-plan persistent launch (sfft_execute_persistent: every
level in one cooperative launch, grid-wide barriers between levels) writes
the ciphertexts of the launch-per-level execution, bit for bit, on small
plans of several shapes, twice in a row, with no barrier wait running out;
a geometry it does not serve is refused before anything runs."""
import sys

import numpy as np
import pytest
import torch

from paper_1611_08769_amd import api
from paper_1611_08769_amd import sfft as S

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(1, 8, 8, 4, False), (1, 4, 8, 4, True), (2, 4, 8, 4, False), (1, 16, 12, 6, True)],
                         ids=str)
def test_persistent_matches_per_level_launches(shape):
    dims, L, F, f, cplx = shape
    print("[gpu-case] persistent", shape, flush=True)
    sys.stdout.flush()
    rng = np.random.default_rng(L + 3 * dims)
    pts = L if dims == 1 else L * L
    words = rng.integers(-(1 << (F - 1)), 1 << (F - 1), pts * (2 if cplx else 1)).astype(np.int64)
    p = api.size_params(dims, L, F, f, cplx, 1)
    keys = api.keygen(p, 13)
    ct_in = api.encrypt_words(keys, words, F, seed=13)
    plan = api.Plan(dims, L, F, f, cplx, p)
    want = plan.execute(ct_in).clone()
    for rep in range(2):
        got = torch.zeros_like(want)
        plan.execute_persistent(ct_in, got)
        torch.cuda.synchronize()
        assert S.sfft_plan_persistent_timeouts(plan.handle) == 0
        assert torch.equal(got, want), rep
    plan.close()


def test_persistent_512_thread_body():
    # n = 1, k = 640: Nct = 1280 rows of 160 bytes, too many chunks for the
    # LDS of the 256-thread body, so the 512-thread body runs the products
    print("[gpu-case] persistent 512-thread body", flush=True)
    sys.stdout.flush()
    p = S.params(1, 640)
    words = np.random.default_rng(5).integers(-128, 128, 8).astype(np.int64)
    keys = api.keygen(p, 17)
    ct_in = api.encrypt_words(keys, words, 8, seed=17)
    plan = api.Plan(1, 4, 8, 4, True, p)
    want = plan.execute(ct_in).clone()
    got = torch.zeros_like(want)
    plan.execute_persistent(ct_in, got)
    torch.cuda.synchronize()
    assert S.sfft_plan_persistent_timeouts(plan.handle) == 0
    assert torch.equal(got, want)
    plan.close()


def test_persistent_refuses_wide_rows():
    # n = 3, k = 704: rows of 352 bytes, 11 fragments
    p = S.params(3, 704)
    plan = api.Plan(1, 2, 4, 2, True, p)
    ct_in = torch.zeros((plan.info.n_inputs, plan.ct_words), dtype=torch.int32, device="cuda")
    with pytest.raises(S.SfftError) as ei:
        plan.execute_persistent(ct_in)
    assert ei.value.code == S.SFFT_EUNSUPPORTED
    plan.close()
