"""tg_count_batch_noalloc (no device allocation; scratch in a fixed device
array) against tg_count_batch: two calls in a row, the second with fewer
and smaller graphs, both bit-exact, plus the size limit."""
import ctypes

import numpy as np
import pytest

import graphgen
from _gpu import device, note

pytestmark = pytest.mark.gpu


def _args(b):
    import torch

    import paper_1901_10026_amd as tg
    dev = device()
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)
    return (t(b.node_off, np.int64), t(b.slot_off, np.int64), t(b.row_ptr, np.int32), t(b.col_idx, np.int32),
            t(b.types, np.uint8), t(b.L, np.uint8), t(tg.key_offsets(b.L), np.int64))


def test_noalloc_batch_equals_batch_twice():
    import torch

    import paper_1901_10026_amd as tg
    big = graphgen.batch_gnp(3000, 1, 500, 0.02, 0.4, 1, 8, 61)
    small = graphgen.batch_gnp(400, 1, 120, 0.05, 0.5, 1, 8, 62)
    for name, b in (("first call, 3000 graphs", big), ("second call, 400 smaller graphs", small)):
        a = _args(b)
        got = tg.count_batch(*a, noalloc=True)
        torch.cuda.synchronize()
        want = tg.count_batch(*a)
        torch.cuda.synchronize()
        note(f"{name}: {b.G} graphs, {int(b.slot_off[-1]) // 2} edges")
        assert torch.equal(got.view(torch.int64), want.view(torch.int64)), name
    # and the no-allocation call again on the first batch after the second
    a = _args(big)
    again = tg.count_batch(*a, noalloc=True)
    want = tg.count_batch(*a)
    torch.cuda.synchronize()
    assert torch.equal(again.view(torch.int64), want.view(torch.int64))


def test_noalloc_batch_rejects_too_many_graphs():
    import paper_1901_10026_amd as tg
    b = graphgen.batch_gnp(4, 3, 10, 0.3, 0.5, 1, 3, 63)
    a = _args(b)
    out = tg.count_batch(*a)
    opt = tg._Options()
    tg.lib().tg_options_default(ctypes.byref(opt))
    st = tg.lib().tg_count_batch_noalloc((1 << 21) + 1, *[x.data_ptr() for x in a], out.data_ptr(),
                                         ctypes.byref(opt), None)
    assert st == 1 and b"at most" in tg.lib().tg_last_error()
