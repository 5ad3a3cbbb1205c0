"""The allocation-free Mult (hs_mult_relin_noalloc: raw device buffers in and
out, every intermediate in the library's fixed scratch array) against
hs_mult_relin on the same ciphertexts: the output words must be identical,
on two calls in a row, the second with a smaller input (a lower level), with
and without rescale; and its refusals (a level whose intermediates exceed the
scratch, tables not built yet, bad pointers)."""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

LEVELS = {"toy12": (23, 6), "fgb16": (12, 3)}


def _dev(words):
    """host uint64 words -> a CUDA int64 tensor holding the same bits"""
    import torch
    return torch.from_numpy(np.ascontiguousarray(words).reshape(-1).view(np.int64).copy()).cuda()


def _host(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.fixture(scope="module", params=sorted(LEVELS))
def ctx(request):
    from paper_2410_11184_amd import hs
    c = hs.Context(synthetic.preset(request.param), device=0, stream=hs.current_stream())
    c.keygen(31)
    return request.param, c


def _pair(c, level, seed):
    r = np.random.default_rng(seed)
    za = r.uniform(-1, 1, c.slots)
    zb = r.uniform(-1, 1, c.slots)
    return c.encrypt(za, level, c.delta, seed), c.encrypt(zb, level, c.delta, seed + 1)


@pytest.mark.parametrize("rescale", [True, False])
def test_matches_mult_relin_on_two_calls(ctx, rescale):
    import torch
    name, c = ctx
    for i, level in enumerate(LEVELS[name]):
        a, b = _pair(c, level, 100 * i + (7 if rescale else 0))
        ref = c.mult(a, b, rescale=rescale)             # also builds this level's key-switching tables
        want = ref.export()
        da, db = _dev(a.export()), _dev(b.export())
        out = torch.empty(want.size, dtype=torch.int64, device="cuda")
        print("noalloc mult: %s level %d rescale %s" % (name, level, rescale), flush=True)
        s = c.mult_noalloc(da.data_ptr(), db.data_ptr(), level, a.scale, b.scale, out.data_ptr(), rescale=rescale)
        c.sync()
        torch.cuda.synchronize()
        got = _host(out).reshape(want.shape)
        assert s == ref.scale, (level, s, ref.scale)
        bad = np.argwhere(got != want)
        assert bad.size == 0, "level %d: %d words differ, first %s" % (level, len(bad), bad[:1])


def test_refusals(ctx):
    import torch
    from paper_2410_11184_amd import hs
    name, c = ctx
    level = LEVELS[name][1]
    a, b = _pair(c, level, 5)
    c.mult(a, b)
    da, db = _dev(a.export()), _dev(b.export())
    out = torch.empty(da.numel(), dtype=torch.int64, device="cuda")
    with pytest.raises(hs.HSError) as e:             # out overlapping an input
        c.mult_noalloc(da.data_ptr(), db.data_ptr(), level, a.scale, b.scale, da.data_ptr())
    assert e.value.name == "HS_E_ARG"
    with pytest.raises(hs.HSError) as e:             # misaligned
        c.mult_noalloc(da.data_ptr() + 8, db.data_ptr(), level, a.scale, b.scale, out.data_ptr())
    assert e.value.name == "HS_E_ARG"
    with pytest.raises(hs.HSError) as e:
        c.mult_noalloc(da.data_ptr(), db.data_ptr(), c.nq, a.scale, b.scale, out.data_ptr())
    assert e.value.name == "HS_E_LEVEL"
    if name == "fgb16":
        # level 20 of the N = 2^16 chain: ~148 MiB of intermediates (checked
        # before any pointer is used, so these buffers need not be that large)
        with pytest.raises(hs.HSError) as e:
            c.mult_noalloc(da.data_ptr(), db.data_ptr(), 20, a.scale, b.scale, out.data_ptr())
        assert e.value.name == "HS_E_ARG"


def test_tables_must_exist_first():
    import torch
    from paper_2410_11184_amd import hs
    c = hs.Context(synthetic.preset("toy12"), device=0, stream=hs.current_stream())
    c.keygen(32)
    a, b = _pair(c, 15, 9)
    da, db = _dev(a.export()), _dev(b.export())
    out = torch.empty(da.numel(), dtype=torch.int64, device="cuda")
    with pytest.raises(hs.HSError) as e:
        c.mult_noalloc(da.data_ptr(), db.data_ptr(), 15, a.scale, b.scale, out.data_ptr())
    assert e.value.name == "HS_E_STATE"
