"""The no-allocation trust check (gx_sn_check_noalloc) against the allocating
one (gx_sn_check), through the C ABI: two calls in a row, the second with
fewer regions and a smaller grid (the static scratch keeps the first call's
flags, which must not leak into the second), the empty call, and the size
limit of the static scratch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _pred(rng, k, grid, lo, hi):
    v = rng.uniform(lo, hi, size=(k, grid ** 3, 5)).astype(np.float32)
    return v


def test_noalloc_check_matches_allocating_check(gx):
    import torch
    eng = gx.Engine(0)
    try:
        lo = np.array([-1.0, 0.0, -2.0, -3.0, 1.0])
        hi = np.array([1.0, 5.0, 2.0, 3.0, 2.0])
        rng = np.random.default_rng(41)
        # first call: 9 regions on a 12^3 grid with planted faults
        k1, g1 = 9, 12
        v = _pred(rng, k1, g1, lo, hi)
        v[0, 5, 0] = 1.0001             # above
        v[2, g1 ** 3 - 1, 4] = np.nan   # last value
        v[3, 0, 1] = np.float32(hi[1])  # on the bound: trusted
        v[5, 17, 3] = -np.inf
        v[8, 100, 2] = -2.5             # below
        pred = torch.as_tensor(v.reshape(-1).copy(), device="cuda")
        ref = eng.sn_check(pred, k1, g1, lo, hi)
        ok = torch.full((k1,), 7, dtype=torch.uint8, device="cuda")
        eng.sn_check_noalloc(pred, k1, g1, lo, hi, ok)
        torch.cuda.synchronize()
        assert ref.tolist() == [False, True, False, True, True, False, True, True, False]
        assert ok.cpu().numpy().astype(bool).tolist() == ref.tolist()
        # second call, smaller: 4 regions on an 8^3 grid, all but one trusted;
        # region 0 was faulty in the first call and must now pass
        k2, g2 = 4, 8
        w = _pred(rng, k2, g2, lo, hi)
        w[3, 7, 2] = 2.0001
        pred2 = torch.as_tensor(w.reshape(-1).copy(), device="cuda")
        ref2 = eng.sn_check(pred2, k2, g2, lo, hi)
        ok2 = torch.full((k2,), 7, dtype=torch.uint8, device="cuda")
        eng.sn_check_noalloc(pred2, k2, g2, lo, hi, ok2)
        torch.cuda.synchronize()
        assert ref2.tolist() == [True, True, True, False]
        assert ok2.cpu().numpy().astype(bool).tolist() == ref2.tolist()
        # k = 0 writes nothing
        ok0 = torch.full((1,), 7, dtype=torch.uint8, device="cuda")
        eng.sn_check_noalloc(pred2, 0, g2, lo, hi, ok0)
        torch.cuda.synchronize()
        assert int(ok0.item()) == 7
        # beyond the static scratch: a clear error, nothing launched
        big = gx._lib.GX_NOALLOC_MAX_REGIONS + 1
        with pytest.raises(gx.GxError, match="static scratch"):
            eng.sn_check_noalloc(pred2, big, g2, lo, hi, ok2)
    finally:
        eng.close()
